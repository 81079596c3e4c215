"""RK34 pseudo-time stepping with locally adaptive pseudo-steps -- TEST
INFRASTRUCTURE ONLY (part of the oracle).

Sec. 5 runs its pseudo-iterations with an embedded RK34 pair and locally
adaptive pseudo-steps (citing earlier work for both); it prints neither the
coefficients nor the controller.  Readings taken here:
  * the pair is Kennedy, Carpenter and Lewis's four-stage, third-order,
    two-register scheme with an embedded second-order solution
    (RK3(2)4[2R+]C): stage i uses U + sum_{j < i-1} b_j h k_j + a_{i,i-1} h k_{i-1};
  * h is a field: one pseudo-step per state value;
  * after each step every value's step is scaled by
        clamp(SAFETY * (|e| / atol)^(-1/3), FAC_MIN, FAC_MAX),
    e = h sum_j (b_j - bhat_j) k_j the embedded error estimate, atol the
    convergence tolerance, and kept within [h0 / MULT, MULT h0] of the initial
    pseudo-step h0.
Pins: tests/test_oracle_rk34.py.
"""
import numpy as np

# RK3(2)4[2R+]C (Kennedy, Carpenter, Lewis 2000)
A21 = 11847461282814 / 36547543011857
A32 = 3943225443063 / 7078155732230
A43 = -346793006927 / 4029903576067
B = np.array([1017324711453 / 9774461848756, 8237718856693 / 13685301971492,
              57731312506979 / 19404895981398, -101169746363290 / 37734290219643])
BHAT = np.array([15763415370699 / 46270243929542, 514528521746 / 5659431552419,
                 27030193851939 / 9429696342944, -69544964788955 / 30262026368149])
SAFETY, FAC_MIN, FAC_MAX, MULT = 0.8, 0.98, 1.01, 3.0


def butcher():
    """Full Butcher matrix of the two-register scheme."""
    A = np.zeros((4, 4))
    A[1, 0] = A21
    A[2, 0], A[2, 1] = B[0], A32
    A[3, 0], A[3, 1], A[3, 2] = B[0], B[1], A43
    return A


def step(rhs, U, h, h0, atol):
    """One RK34 step of dU/dtau = rhs(U) with the step field h; returns the new
    state and the new step field."""
    A = butcher()
    ks = []
    for i in range(4):
        Ui = U + h * sum(A[i, j] * ks[j] for j in range(i)) if i else U
        ks.append(rhs(Ui))
    Unew = U + h * sum(B[j] * ks[j] for j in range(4))
    e = h * sum((B[j] - BHAT[j]) * ks[j] for j in range(4))
    err = np.maximum(np.abs(e) / atol, 1e-300)
    fac = np.clip(SAFETY * err ** (-1.0 / 3.0), FAC_MIN, FAC_MAX)
    return Unew, np.clip(h * fac, h0 / MULT, h0 * MULT)
