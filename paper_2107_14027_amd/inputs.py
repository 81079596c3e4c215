"""Seeded synthetic inputs for the ACM-HD flux-reconstruction residual.

This module only builds input arrays (closed-form fields sampled at the
solution points, plus seeded noise); it contains none of the method's
arithmetic and is shared by the tests, the benchmark and the smoke check so
that the GPU library and the CPU oracle see identical inputs.

State layout: U[e][v][k][j][i] as float64, e = ex + nx*(ey + ny*ez), i fastest,
v in [P, u, v, w, q_x, q_y, q_z, r_x, r_y, r_z, s_x, s_y, s_z] with
q = grad u, r = grad v, s = grad w.  Solution points are the Gauss-Legendre
nodes (taken from numpy.polynomial.legendre.leggauss) of each element.

Fields (Sec. 5 of the paper defines the Taylor-Green vortex on [0, 2 pi]^3):
  tgv       u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
            P = P0 + (1/16)(cos 2x + cos 2y)(cos 2z + 2), aux = exact gradients
  fourier   random Fourier velocity and pressure, |k|_2 <= kmax, unit RMS
  sines     P = u = v = w = sin x sin y sin z, aux = exact gradients
Meshes of linear hexahedra (corner lists, seeded vertex displacements) come
from linear_hex_corners.
"""
import numpy as np

NV = 13
NAMES = ("P", "u", "v", "w", "qx", "qy", "qz", "rx", "ry", "rz", "sx", "sy", "sz")


def box_jacobian(n):
    """dx/dxi of the uniform lattice of the periodic box [0, 2 pi]^3 (row-major 3x3)."""
    nx, ny, nz = n
    return np.diag([np.pi / nx, np.pi / ny, np.pi / nz])


def nodes(p):
    return np.polynomial.legendre.leggauss(p + 1)


def point_coords(p, n, jac=None):
    """Physical coordinates X[e][3][m^3] of every solution point.

    The element with lattice index (ex, ey, ez) is the image of [-1, 1]^3 under
    x = J (xi + 1 + 2 (ex, ey, ez))."""
    nx, ny, nz = n
    m = p + 1
    J = box_jacobian(n) if jac is None else np.asarray(jac, dtype=np.float64).reshape(3, 3)
    xi, _ = nodes(p)
    kk, jj, ii = np.meshgrid(xi, xi, xi, indexing="ij")          # [k][j][i]
    ref = np.stack([ii.ravel(), jj.ravel(), kk.ravel()])          # [3][m^3]
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    org = np.stack([ex.ravel(), ey.ravel(), ez.ravel()], axis=1)  # [ne][3]
    local = ref[None, :, :] + 1.0 + 2.0 * org[:, :, None]         # [ne][3][m^3]
    return np.einsum("ab,ebq->eaq", J, local)


def _assemble(P, V, G):
    """Stack P [e][q], V [3][e][q], G [3][3][e][q] (G[i][k] = d u_i / d x_k)."""
    ne, nq = P.shape
    U = np.empty((ne, NV, nq))
    U[:, 0] = P
    for i in range(3):
        U[:, 1 + i] = V[i]
        for k in range(3):
            U[:, 4 + 3 * i + k] = G[i][k]
    return U


def tgv(p, n, P0=0.0, noise=0.0, seed=20210729, jac=None):
    """Taylor-Green vortex with exact velocity gradients, optional N(0, noise^2) on all 13."""
    X = point_coords(p, n, jac)
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    sx, cx, sy, cy, sz, cz = np.sin(x), np.cos(x), np.sin(y), np.cos(y), np.sin(z), np.cos(z)
    u = sx * cy * cz
    v = -cx * sy * cz
    w = np.zeros_like(u)
    P = P0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    G = [[cx * cy * cz, -sx * sy * cz, -sx * cy * sz],
         [sx * sy * cz, -cx * cy * cz, cx * sy * sz],
         [w, w, w]]
    U = _assemble(P, [u, v, w], G)
    if noise:
        U += np.random.default_rng(seed).normal(0.0, noise, size=U.shape)
    return U


def sines(p, n, jac=None):
    """P = u = v = w = sin x sin y sin z with exact gradients."""
    X = point_coords(p, n, jac)
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    f = np.sin(x) * np.sin(y) * np.sin(z)
    g = [np.cos(x) * np.sin(y) * np.sin(z), np.sin(x) * np.cos(y) * np.sin(z),
         np.sin(x) * np.sin(y) * np.cos(z)]
    return _assemble(f, [f, f, f], [g, g, g])


def _wavevectors(kmax):
    r = np.arange(-kmax, kmax + 1)
    K = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    k2 = (K ** 2).sum(1)
    return K[(k2 > 0) & (k2 <= kmax * kmax)]


def fourier(p, n, seed, kmax=4, device=None):
    """Random smooth periodic field on the box [0, 2 pi]^3 (axis-aligned lattice).

    Each of P, u, v, w is sum_k a_k cos(k.x) + b_k sin(k.x) over integer k with
    0 < |k|_2 <= kmax, a, b ~ N(0, 1), scaled to unit RMS over the solution
    points; the aux variables are the exact velocity gradients.  Evaluated
    separably along the three axes.  With device (a torch device string) the
    same coefficients are synthesised with torch on that device and a float64
    torch tensor is returned; otherwise a numpy array."""
    nx, ny, nz = n
    m = p + 1
    rng = np.random.default_rng(seed)
    K = _wavevectors(kmax)
    xi, _ = nodes(p)
    ax = [np.pi / nd * (xi[None, :] + 1.0 + 2.0 * np.arange(nd)[:, None]).ravel()
          for nd in (nx, ny, nz)]
    ks = np.arange(-kmax, kmax + 1)
    E = [np.exp(1j * ks[:, None] * a[None, :]) for a in ax]       # [2kmax+1][n_d m]
    if device is not None:
        import torch
        lib = torch
        E = [torch.from_numpy(e).to(device) for e in E]
        asarr = lambda a: torch.from_numpy(a).to(device)
        out = torch.empty((nx * ny * nz, NV, m ** 3), dtype=torch.float64, device=device)
        meansq = lambda v: float(torch.mean(v * v))
    else:
        lib = np
        asarr = lambda a: a
        out = np.empty((nx * ny * nz, NV, m ** 3))
        meansq = lambda v: float(np.mean(v * v))

    def synth(coef):
        # coef: complex [2kmax+1]^3 spectrum; field = Re sum c e^{i k.x}
        t = lib.einsum("abc,cz->abz", coef, E[2])
        t = lib.einsum("abz,by->ayz", t, E[1])
        t = lib.einsum("ayz,ax->zyx", t, E[0])
        return t.real                                            # [Z][Y][X]

    def to_layout(F):
        F = F.reshape(nz, m, ny, m, nx, m)                        # [ez][k][ey][j][ex][i]
        return F.permute(0, 2, 4, 1, 3, 5).reshape(nx * ny * nz, m ** 3) if device is not None \
            else F.transpose(0, 2, 4, 1, 3, 5).reshape(nx * ny * nz, m ** 3)

    idx = tuple((K + kmax).T)
    for f in range(4):
        a = rng.standard_normal(len(K))
        b = rng.standard_normal(len(K))
        coef = np.zeros((2 * kmax + 1,) * 3, dtype=np.complex128)
        # a cos + b sin = Re[(a - i b) e^{i k.x}]
        np.add.at(coef, idx, a - 1j * b)
        val = synth(asarr(coef))
        scale = 1.0 / np.sqrt(meansq(val))
        out[:, f] = to_layout(val) * scale
        if f >= 1:
            for kdir in range(3):
                dc = np.zeros_like(coef)
                np.add.at(dc, idx, 1j * K[:, kdir] * (a - 1j * b))
                out[:, 4 + 3 * (f - 1) + kdir] = to_layout(synth(asarr(dc))) * scale
    return out


def uniform(p, n, values):
    """Uniform state with the 13 given values."""
    nx, ny, nz = n
    m = p + 1
    U = np.empty((nx * ny * nz, NV, m ** 3))
    U[:] = np.asarray(values, dtype=np.float64)[None, :, None]
    return U


def noise(shape, sigma, seed):
    return np.random.default_rng(seed).normal(0.0, sigma, size=shape)


def nu_T_from_length(Re, Lr):
    """nu = 1/Re; relaxation time T = Lr^2 / nu for a relaxation length Lr."""
    nu = 1.0 / Re
    return nu, Lr * Lr / nu


def linear_hex_corners(n, amp=0.0, seed=0, smooth=0.0):
    """Corner coordinates C[e][8][3] of a periodic lattice of linear hexahedra
    filling [0, 2 pi]^3 (corner c = c0 + 2 c1 + 4 c2, c_d = 0 at xi_d = -1).
    Vertex (i, j, k) sits at 2 pi (i/nx, j/ny, k/nz) moved by
      amp * h * uniform(-1, 1)^3            (seeded, periodic in the vertex lattice)
      + smooth * (sin y sin z, sin z sin x, sin x sin y)   at the undisplaced position,
    h the smallest element width.  Each element stores its own corners, with
    2 pi added across the periodic seam, so elements sharing a face store the
    same face up to that shift."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    h = 2 * np.pi / max(n)
    disp = amp * h * rng.uniform(-1.0, 1.0, size=(nz, ny, nx, 3))
    e = np.arange(nx * ny * nz)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    C = np.empty((len(e), 8, 3))
    for c in range(8):
        cx, cy, cz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        ix, iy, iz = ex + cx, ey + cy, ez + cz
        X = np.stack([2 * np.pi * ix / nx, 2 * np.pi * iy / ny, 2 * np.pi * iz / nz], axis=1)
        X = X + disp[iz % nz, iy % ny, ix % nx]
        x0, y0, z0 = (2 * np.pi * ix / nx, 2 * np.pi * iy / ny, 2 * np.pi * iz / nz)
        X[:, 0] += smooth * np.sin(y0) * np.sin(z0)
        X[:, 1] += smooth * np.sin(z0) * np.sin(x0)
        X[:, 2] += smooth * np.sin(x0) * np.sin(y0)
        C[:, c] = X
    return C


def linear_hex_points(p, C):
    """Physical coordinates x[e][3][m^3] of the solution points of linear
    hexahedra with corners C[e][8][3] (trilinear interpolation of the corners)."""
    m = p + 1
    xg, _ = nodes(p)
    q = np.arange(m ** 3)
    xi = np.stack([xg[q % m], xg[(q // m) % m], xg[q // (m * m)]], axis=1)   # [m^3][3]
    out = np.zeros((C.shape[0], 3, m ** 3))
    for c in range(8):
        s = np.array([2 * (c & 1) - 1, 2 * ((c >> 1) & 1) - 1, 2 * ((c >> 2) & 1) - 1])
        N = np.prod(0.5 * (1 + s[None, :] * xi), axis=1)                       # [m^3]
        out += C[:, c, :, None] * N[None, None, :]
    return out
