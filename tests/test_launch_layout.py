"""Host-side checks of the fused kernels' launch invariants, with the launch
shapes the library reports (fr_launch_shape, no device work): LDS fits a
compute unit, the per-batch neighbour
table is fully covered by the workgroup's threads, every receiving trace
block is written by exactly one (element, face), and every staged read lies
inside the trace array.  These mirror the index formulas of k_trace and
k_fused (face f = 2d + side, neighbour across a face, padded trace blocks)."""
import pytest

from paper_2107_14027_amd import binding as B

NV, NTR, LDS_BYTES = 13, 7, 160 * 1024
PREC = {"D": B.FR_F64, "F": B.FR_F32}


def shapes(p, prec):
    """(trace E, trace threads, trace LDS), (fused E, fused threads, fused LDS)."""
    return (B.fr_launch_shape(p, PREC[prec], B.FR_K_TRACE),
            B.fr_launch_shape(p, PREC[prec], B.FR_K_FUSED))


def neighbour(e, f, nx, ny, nz):
    ex, r = e % nx, e // nx
    ey, ez = r % ny, r // ny
    d, up = f >> 1, f & 1
    step = 1 if up else -1
    if d == 0:
        ex = (ex + step) % nx
    elif d == 1:
        ey = (ey + step) % ny
    else:
        ez = (ez + step) % nz
    return ex + nx * (ey + ny * ez)


def layout(p, prec):
    esz = 8 if prec == "D" else 4
    m = p + 1
    w = 16 // esz
    chp = (NTR * m * m + w - 1) // w * w
    return esz, m, chp, chp // w


@pytest.mark.parametrize("prec", ["D", "F"])
@pytest.mark.parametrize("p", range(1, 7))
def test_lds_fits(p, prec):
    esz, m, chp, _ = layout(p, prec)
    ns = m ** 3
    (te, tnt, tlds), (e, nt, lds) = shapes(p, prec)
    mp = m + 1 if (m % 2 == 0 and m >= 4) else m        # padded x-line pitch of k_trace
    assert tlds == (te * NV * mp * m * m + 2 * m) * esz + 6 * te * 4 <= LDS_BYTES
    assert lds == (e * (NV + 9) * ns + 6 * e * chp + m * m + 4 * m + 24) * esz <= LDS_BYTES
    assert nt % 64 == 0 and tnt % 64 == 0 and nt >= 2 * m and tnt >= 2 * m


LATTICES = [(5, 3, 4), (1, 1, 1), (2, 1, 1), (1, 2, 3), (4, 4, 4), (3, 5, 2)]


@pytest.mark.parametrize("prec", ["D", "F"])
@pytest.mark.parametrize("p", range(1, 7))
def test_trace_blocks_written_once_and_reads_in_range(p, prec):
    _, _, _, chv = layout(p, prec)
    (temax, tnt, _), (emax, nt, _) = shapes(p, prec)
    for nx, ny, nz in LATTICES:
        ne = nx * ny * nz
        te = min(temax, ne)
        written = {}
        for b in range((ne + te - 1) // te):
            e0 = b * te
            nel = min(te, ne - e0)
            covered = {t for tid in range(tnt) for t in range(tid, 6 * nel, tnt)}
            assert covered == set(range(6 * nel))          # neighbour table fully filled
            for t in range(6 * temax * chv):
                f, r = divmod(t, temax * chv)
                el, k = divmod(r, chv)
                if el < nel:
                    nb = neighbour(e0 + el, f, nx, ny, nz)
                    idx = ((f ^ 1) * ne + nb) * chv + k
                    written[idx] = written.get(idx, 0) + 1
        assert sorted(written) == list(range(6 * ne * chv)) and set(written.values()) == {1}
        e = min(emax, ne)
        run, nch = emax * chv, 6 * emax * chv
        for b in range((ne + e - 1) // e):
            e0 = b * e
            nel = min(e, ne - e0)
            for k in range(nch):
                f, o = divmod(k, run)
                if nel == emax or o < nel * chv:
                    assert 0 <= (f * ne + e0) * chv + o < 6 * ne * chv


def test_launch_shape_rejects_bad_arguments():
    for args in ((0, B.FR_F64, B.FR_K_FUSED), (7, B.FR_F64, B.FR_K_FUSED), (3, 2, B.FR_K_FUSED),
                 (3, B.FR_F64, 2)):
        with pytest.raises(B.FrError):
            B.fr_launch_shape(*args)
