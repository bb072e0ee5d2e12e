"""CPU emulation of the lane exchanges of the operator-resident kernels
(FP32 and FP64 forms): the DPP partner patterns inside a 16-lane row, the
register row order i -> i ^ s(p), the halving row sums, the row gather, and
the permlane16 / permlane32 swap levels of the column sums, with their
column offsets.  Run on integer-valued data (exact in FP64), one workgroup's
tiles of Avs, every tile shape the kernels instantiate: the emulated
exchanges must give exactly Avs S (every lane's owned row) and the wave's
column sums of Avs^T V (every lane's quarter of its columns).  Host logic
only: no GPU, no library.

The instruction semantics emulated (checked on the device by the parity
tests of both kernels): row_ror:8 reads lane (p + 8) mod 16 of the row,
row_half_mirror lane (p & 8) | (7 - (p & 7)), quad_perm [2,3,0,1] lane
p ^ 2, quad_perm [1,0,3,2] lane p ^ 1; v_permlane16_swap(a, b) exchanges b
of each even 16-lane row with a of the odd row above it, v_permlane32_swap
the same between the two 32-lane halves.
"""
import numpy as np
import pytest


def ror8(p):
    return (p + 8) % 16


def half_mirror(p):
    return (p & 8) | (7 - (p & 7))


PARTNERS = [ror8, half_mirror, lambda p: p ^ 2, lambda p: p ^ 1]


def row_xor(TR, p):
    b3, b2, b1 = (p >> 3) & 1, (p >> 2) & 1, (p >> 1) & 1
    if TR == 8:
        return 4 * b3 + 2 * b2 + (b1 ^ b2)
    if TR == 4:
        return 2 * b3 + b2
    return b3


def col_off(TC, rho):
    return (rho & 1) * (TC // 2) + (rho >> 1) * (TC // 4)


def row_sum(acc):
    """acc: (16, TR) partials of one 16-lane row; returns (16,) acc[0]."""
    acc = acc.copy()
    TR = acc.shape[1]
    for level, part in enumerate(PARTNERS):
        H = TR >> (level + 1)
        src = np.array([part(p) for p in range(16)])
        if H >= 1:
            acc[:, :H] = acc[:, :H] + acc[src, H:2 * H]
        else:
            acc[:, 0] = acc[:, 0] + acc[src, 0]
    return acc[:, 0]


def row_gather(x, TR):
    """x: (16,) value per lane; returns (16, TR), vv[p, i] = x of a lane p'
    with s(p') = s(p) ^ i."""
    vv = np.zeros((16, TR))
    vv[:, 0] = x
    mv = lambda a, f: a[np.array([f(p) for p in range(16)])]
    if TR == 8:
        vv[:, 4] = mv(vv[:, 0], ror8)
        vv[:, 2] = mv(vv[:, 0], half_mirror)
        vv[:, 6] = mv(vv[:, 4], half_mirror)
        for i in range(0, 8, 2):
            vv[:, i + 1] = mv(vv[:, i], lambda p: p ^ 2)
    elif TR == 4:
        vv[:, 2] = mv(vv[:, 0], ror8)
        vv[:, 1] = mv(vv[:, 0], half_mirror)
        vv[:, 3] = mv(vv[:, 2], half_mirror)
    else:
        vv[:, 1] = mv(vv[:, 0], ror8)
    return vv


def permlane_swap(a, b, width):
    """Per lane of a wave: a, b (64,) -> the two results (a', b'): b of the
    lower block of each 2 x width pair is exchanged with a of the upper."""
    a2, b2 = a.copy(), b.copy()
    for l in range(64):
        if (l // width) % 2 == 0:
            u = l + width
            a2[u], b2[l] = b[l], a[u]
    return a2, b2


def col_sum_rows(q):
    """q: (64, TC) column partials per lane of a wave; returns (64, TC // 4)."""
    q = q.copy()
    TC = q.shape[1]
    H1, H2 = TC // 2, TC // 4
    for j in range(H1):
        r0, r1 = permlane_swap(q[:, j], q[:, j + H1], 16)
        q[:, j] = r0 + r1
    for j in range(H2):
        r0, r1 = permlane_swap(q[:, j], q[:, j + H2], 32)
        q[:, j] = r0 + r1
    return q[:, :H2]


@pytest.mark.parametrize("TR,TC", [(2, 4), (2, 16), (4, 4), (4, 8), (8, 4), (8, 8), (8, 12), (8, 16)])
def test_resident_exchanges_reproduce_the_products(TR, TC):
    rng = np.random.default_rng(TR * 100 + TC)
    KV, KS = 4 * TR, 16 * TC                # four row blocks (one wave) x 16 column blocks
    A = rng.integers(-8, 9, (KV, KS)).astype(np.float64)
    S = rng.integers(-8, 9, KS).astype(np.float64)
    V = rng.integers(-8, 9, KV).astype(np.float64)
    q = np.zeros((64, TC))
    for rho in range(4):                    # the four 16-lane rows of the wave
        rb = rho
        acc = np.zeros((16, TR))
        for p in range(16):
            sx = row_xor(TR, p)
            for i in range(TR):
                r = TR * rb + (i ^ sx)
                acc[p, i] = A[r, TC * p:TC * p + TC] @ S[TC * p:TC * p + TC]
        rs = row_sum(acc)
        for p in range(16):
            r = TR * rb + row_xor(TR, p)
            assert rs[p] == A[r] @ S, (rho, p)          # every lane: the full sum of its owned row
        # the stress operand: the gathered rows in register order
        own = np.array([V[TR * rb + row_xor(TR, p)] for p in range(16)])
        vv = row_gather(own, TR)
        for p in range(16):
            sx = row_xor(TR, p)
            for i in range(TR):
                assert vv[p, i] == V[TR * rb + (i ^ sx)]
            for j in range(TC):
                c = TC * p + j
                q[16 * rho + p, j] = sum(A[TR * rb + (i ^ sx), c] * vv[p, i] for i in range(TR))
    if TC % 4 == 0:
        wave = col_sum_rows(q)
        colsum = A.T @ V                     # the wave's rows are all of A here
        for l in range(64):
            rho, p = l >> 4, l & 15
            for j in range(TC // 4):
                assert wave[l, j] == colsum[TC * p + col_off(TC, rho) + j], (l, j)
