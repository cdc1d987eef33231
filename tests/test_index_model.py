"""Host model of the row-packed TSMM kernel's index arithmetic and of the
leap-frog register ring, stepped tile by tile on the CPU.

The model follows tsmm_packed (csrc/tsg_kernels.hpp) and leapfrog_ring /
leapfrog (csrc/tsg_device.hpp) lane by lane: which rows and columns each lane
loads into which register set of the ring, which set each multiplication
reads, how v_mfma_f64_16x16x4f64 combines the lanes' operands (lane l
supplies A(l % 16, l / 16) and B(l / 16, l % 16); element r of lane l is
D(l / 16 + 4 r, l % 16)), and where each output lane stores.  On integer
data the modelled launch must reproduce A C exactly, write every output
element exactly once, touch no address outside A, and multiply only the
register set that holds the tile being computed -- on grids of three blocks
that work through many tiles, the case in which the spilled complex 15 x 15
variant with four register sets went wrong on the GPU.  The model passing
for that configuration clears the kernel's indexing and the ring rotation
as the cause of that failure.
"""
import numpy as np
import pytest


def ring_schedule(t0, ntiles, G, nbuf):
    """(tile, set) pairs in the order the leap-frog driver loads and computes,
    as events ('load', tile, set) and ('compute', tile, set)."""
    ev = []
    if t0 >= ntiles:
        return ev
    if nbuf == 2:   # leapfrog: two sets used in turn
        x, y = 0, 1
        t = t0
        ev.append(("load", t, x))
        while True:
            t1 = t + G
            if t1 >= ntiles:
                ev.append(("compute", t, x))
                return ev
            ev.append(("load", t1, y))
            ev.append(("compute", t, x))
            t2 = t1 + G
            if t2 >= ntiles:
                ev.append(("compute", t1, y))
                return ev
            ev.append(("load", t2, x))
            ev.append(("compute", t1, y))
            t = t2
    last = ntiles - 1 - ((ntiles - 1 - t0) % G)
    for i in range(nbuf - 1):
        ti = t0 + i * G
        ev.append(("load", min(ti, last), i))
    t = t0
    while True:
        for p in range(nbuf):
            ta = t + (nbuf - 1) * G
            ev.append(("load", min(ta, last), (p + nbuf - 1) % nbuf))
            ev.append(("compute", t, p))
            t += G
            if t > last:
                return ev


def model_tsmm_packed(A, C, M, N, U, WPB, NBUF, grid):
    """B = A C as the row-packed kernel computes it (integer data, exact)."""
    K = A.shape[0]
    P = 16 // N
    QN = P * M
    S = (QN + 3) // 4
    RS = 16 * P
    RT = RS * U * WPB
    lanes = np.arange(64)
    lr, lc = lanes >> 4, lanes & 15
    # C operand fragments cf[s, l] = Cop(4 s + l / 16, l % 16)
    cf = np.zeros((S, 64), dtype=A.dtype)
    for s in range(S):
        qq = 4 * s + lr
        hq, m = qq // M, qq % M
        hj, n = lc // N, lc % N
        ok = (qq < QN) & (hj < P) & (hq == hj)
        cf[s, ok] = C[m[ok], n[ok]]
    aok = np.array([[4 * s + r < QN for r in range(4)] for s in range(S)])     # [s, lr]
    B = np.full((K, N), np.nan, dtype=np.complex128 if np.iscomplexobj(A) else np.float64)
    writes = np.zeros((K, N), dtype=np.int64)
    ntiles = (K + RT - 1) // RT
    for b in range(grid):
        for w in range(WPB):
            sets = {}
            for kind, t, p in ring_schedule(b, ntiles, grid, NBUF):
                if kind == "load":
                    frag = np.zeros((U, S, 64), dtype=A.dtype)
                    for u in range(U):
                        r0 = t * RT + (w * U + u) * RS + lc * P
                        for s in range(S):
                            qq = 4 * s + lr
                            ok = aok[s, lr]
                            row = r0 + np.where(ok, qq // M, 0)
                            col = np.where(ok, qq % M, 0)
                            inr = ok & (row < K)
                            addr_row = np.where(inr, row, K - 1)
                            assert np.all((addr_row >= 0) & (addr_row < K) & (col < M)), "load out of A"
                            frag[u, s] = np.where(inr, A[addr_row, col], 0)
                    sets[p] = (t, frag)
                    continue
                loaded_t, frag = sets[p]
                assert loaded_t == t, "set %d holds tile %d, multiplied as tile %d" % (p, loaded_t, t)
                full = (t + 1) * RT <= K
                hj, nj = lc // N, lc % N
                for u in range(U):
                    # D(i, j) = sum_s sum_k Aop_s(i, k) Bop_s(k, j), Aop from lane i + 16 k
                    D = np.zeros((16, 16), dtype=B.dtype)
                    for s in range(S):
                        Aop = frag[u, s].reshape(4, 16).T        # [i, k]
                        Bop = cf[s].reshape(4, 16)              # [k, j]
                        D += Aop @ Bop
                    r0 = t * RT + (w * U + u) * RS + hj
                    for r in range(4):
                        i = lr + 4 * r
                        row = r0 + i * P
                        st = (hj < P) & (full | (row < K))
                        B[row[st], nj[st]] = D[i[st], lc[st]]
                        np.add.at(writes, (row[st], nj[st]), 1)
    return B, writes


CONFIGS = [
    # (M, N, U, WPB, NBUF, complex): the failing spilled variant first
    (15, 15, 2, 4, 4, True), (15, 15, 4, 8, 4, True), (15, 15, 1, 8, 4, True),
    (13, 7, 2, 8, 4, True), (8, 8, 4, 4, 2, False), (3, 5, 2, 8, 4, False), (1, 1, 4, 4, 4, False),
    (16, 16, 2, 4, 3, True), (5, 3, 1, 4, 3, False),
]


@pytest.mark.parametrize("M,N,U,WPB,NBUF,cplx", CONFIGS)
def test_packed_tsmm_index_model(M, N, U, WPB, NBUF, cplx):
    rng = np.random.default_rng([M, N, U, NBUF])
    P = 16 // N
    RT = 16 * P * U * WPB
    K = 3 * RT * 5 + 37            # three blocks, five or six tiles each, ragged tail
    A = rng.integers(-8, 9, (K, M)).astype(np.float64)
    C = rng.integers(-8, 9, (M, N)).astype(np.float64)
    if cplx:
        A = A + 1j * rng.integers(-8, 9, (K, M))
        C = C + 1j * rng.integers(-8, 9, (M, N))
    B, writes = model_tsmm_packed(A, C, M, N, U, WPB, NBUF, grid=3)
    assert np.all(writes == 1), "every output element is written exactly once"
    assert np.array_equal(B, A @ C)


@pytest.mark.parametrize("nbuf", [2, 3, 4])
@pytest.mark.parametrize("t0,ntiles,G", [(0, 17, 3), (2, 17, 3), (1, 2, 3), (0, 1, 1), (5, 40, 7)])
def test_ring_computes_every_tile_once_from_its_own_set(nbuf, t0, ntiles, G):
    ev = ring_schedule(t0, ntiles, G, nbuf)
    held = {}
    done = []
    for kind, t, p in ev:
        if kind == "load":
            assert 0 <= t < ntiles
            held[p] = t
        else:
            assert held[p] == t
            done.append(t)
    assert done == list(range(t0, ntiles, G))
