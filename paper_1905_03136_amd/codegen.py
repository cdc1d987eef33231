"""Code generator: one gfx950 kernel variant per (operation, dtype, M, N).

Section 2.1 of the paper argues for generating the code of every matrix size
instead of writing one generic kernel: with the widths known at compile time
the small loops unroll completely, the accumulators become plain registers and
guard statements remain only where a tile does not divide the width.  Here the
kernel bodies are HIP templates (``csrc/tsg_kernels.hpp``) whose widths are
template arguments; this module decides the configuration of each variant
(mapping, tile, rows in flight, waves per block), writes the explicit
instantiations with their launchers and a registry table, and is run by the
build before compiling.  Widths that are not pre-generated are served by
run-time-width variants of the same templates, which keep the guards.

A configuration can be overridden by the autotuner's table (``tuned.json``).
"""
import json
import math
import os

# storage types of the tall matrices: (ABI id, complex).  r32 / c64 are the
# precision form with binary64 arithmetic on the widened values; r32a / c64a
# the precision form with binary32 products summed in binary32 over stretches
# of 32 rows (binary64 beyond), whose kernels may also be the binary64-
# arithmetic ones of r32 / c64 (more accurate) where those are faster.
DTYPES = {"r64": (0, False), "c128": (1, True), "r32": (2, False), "c64": (3, True),
          "r32a": (4, False), "c64a": (5, True)}
F32_DTYPES = ("r32", "c64", "r32a", "c64a")
A32_DTYPES = ("r32a", "c64a")
# binary64-arithmetic storage twin of a binary32-arithmetic type
A32_TWIN = {"r32a": "r32", "c64a": "c64"}
OPS = {"tsmttsm": 0, "tsmm": 1}

# widths of the plain sweep and the square widths of the target range
GRADED = [(1, 1), (2, 2), (4, 4), (8, 8), (16, 16), (32, 32), (64, 64), (32, 8), (8, 32)]
SQUARE_ALL = [(w, w) for w in range(1, 65)]
# narrow non-square pairs (block vectors of up to eight columns against one
# another): exact-width kernels too, since the run-time-width kernels pad
# them to whole 4-wide slices or 16-column blocks
NARROW = [(m, n) for m in range(1, 9) for n in range(1, 9) if m != n]
# pre-generated widths of the precision form (others use run-time-width variants)
PRECISION = GRADED
# widths whose every candidate the default build compiles into the tuning
# library (the sweep widths and odd pairs with guards on every tile; 17 x 33
# also reaches the LDS-staged kernels with odd complex widths)
TUNE_WIDTHS = GRADED + [(3, 5), (13, 7), (17, 33)]


def is_f32(dt):
    return dt in F32_DTYPES


def is_a32(dt):
    return dt in A32_DTYPES

WPB = 4  # waves per block


def _ceil(a, b):
    return -(-a // b)


# ------------------------------------------------------------ configurations
def _valu_regs(op, M, N, cw, u):
    """Doubles of register state per lane of a VALU variant (accumulators plus
    the two leap-frog operand sets)."""
    if op == "tsmttsm":
        return M * N * cw + 2 * u * (M + N) * cw
    return 2 * u * M * cw + N * cw


def _mfma_regs(op, M, N, cw, c):
    if op == "tsmttsm":
        return c["MB"] * c["NB"] * 4 * cw + 2 * c["U"] * (c["MB"] + c["NB"]) * cw
    return 2 * c["U"] * c["MS"] * cw + c["U"] * c["NB"] * 4 * cw


def candidates(op, dt, M, N):
    """Every configuration the autotuner times for (op, dt, M, N), pruned by
    a register model (the gfx950 analogue of the paper's register estimate
    2 (T_M T_N + 2 (T_M + T_N) + 8), Section 5.2): FP64 operands live in the
    256 architectural VGPRs, MFMA accumulators may use the AGPRs.  The
    binary32-storage types use the matrix-core kinds only; the binary32-
    arithmetic types add the kernels with binary32 products (kind "a32") to
    the candidates of their binary64-arithmetic twin."""
    if is_a32(dt):
        return candidates(op, A32_TWIN[dt], M, N) + _a32_candidates(op, dt, M, N)
    out = _candidates(op, dt, M, N)
    if is_f32(dt):
        out = [c for c in out if c["kind"] != "valu" and not c.get("VA")]
    else:
        out += _lds_candidates(op, dt, M, N)
    return out


LDS_BYTES = 160 * 1024  # LDS of one compute unit (gfx950)


def _lds_candidates(op, dt, M, N):
    """TSMTTSM with the rows staged in LDS by direct loads (tsmttsm_lds) for
    widths above 16: WM x WN waves of MB x NB blocks of 16 x 16 cover C,
    stages of RT rows, two stages in LDS.  Register model in doubles per
    lane: accumulators plus the operands of one stage; two blocks per
    compute unit (OCC = 2) where their LDS fits."""
    out = []
    if op != "tsmttsm" or (M <= 16 and N <= 16):
        return out
    cplx = DTYPES[dt][1]
    cw = 2 if cplx else 1
    # Real odd widths: with K M odd the last element of A shares its 16-byte
    # load with the 8 bytes past the end, and the clamp that keeps that load
    # inside the matrix would move the element (the autotuner's exact-product
    # gate rejected these kernels); complex elements are 16 bytes each.
    if not cplx and (M % 2 or N % 2):
        return out
    mbt, nbt = _ceil(M, 16), _ceil(N, 16)
    for wm in range(1, 9):
        for wn in range(1, 9):
            wpb = wm * wn
            if wpb < 2 or wpb > 8 or wm > mbt or wn > nbt:
                continue
            mb, nb = _ceil(mbt, wm), _ceil(nbt, wn)
            if (wm - 1) * mb >= mbt or (wn - 1) * nb >= nbt:
                continue  # a wave without a block of C
            for g3 in ((0, 1) if cplx else (0,)):
                acc = mb * nb * 4 * (3 if g3 else cw)
                if acc > 64:
                    continue
                for rt in (16, 32, 64):
                    lds = 2 * (_ceil(rt * M * cw, 128) + _ceil(rt * N * cw, 128)) * 128 * 8
                    if lds > LDS_BYTES:
                        continue
                    # IL: operand reads of a stage all at once (0) or IL steps
                    # ahead of the products (then only IL + 1 steps of
                    # operands are live)
                    for il in (0, 1, 2):
                        steps = rt // 4 if il == 0 else min(il + 1, rt // 4)
                        if il and il + 1 > rt // 4:
                            continue
                        ops = steps * (mb + nb) * cw
                        for occ in (1, 2, 3, 4):
                            waves = occ * wpb
                            # the waves of a CU spread evenly over its four SIMDs, at most
                            # three per SIMD, and the register model fits that many
                            if waves % 4 or waves > 12 or occ * lds > LDS_BYTES:
                                continue
                            if acc + ops > (104 if waves <= 8 else 80):
                                continue
                            c = dict(kind="lds", MB=mb, NB=nb, WM=wm, WN=wn, RT=rt, WPB=wpb)
                            if occ > 1:
                                c["OCC"] = occ
                            if g3:
                                c["G3"] = 1
                            if il:
                                c["IL"] = il
                            out.append(c)
    return out


def _lds32_candidates(op, dt, M, N):
    """Binary32-arithmetic TSMTTSM with the rows staged in LDS
    (tsmttsm_lds_a32): as _lds_candidates, stages of 16 or 32 rows (one
    binary32 stretch is 32 rows), rows of whole 16-byte loads.  Register
    model in binary64 units per lane: binary64 sums, binary32 stretch sums
    and live operands (binary32: half a unit each)."""
    out = []
    if op != "tsmttsm" or (M <= 16 and N <= 16):
        return out
    cplx = DTYPES[dt][1]
    cw = 2 if cplx else 1
    if (M * cw) % 4 or (N * cw) % 4:
        return out
    mbt, nbt = _ceil(M, 16), _ceil(N, 16)
    for wm in range(1, 9):
        for wn in range(1, 9):
            wpb = wm * wn
            if wpb < 2 or wpb > 8 or wm > mbt or wn > nbt:
                continue
            mb, nb = _ceil(mbt, wm), _ceil(nbt, wn)
            if (wm - 1) * mb >= mbt or (wn - 1) * nb >= nbt:
                continue
            for g3 in ((0, 1) if cplx else (0,)):
                acc = mb * nb * 4 * cw + mb * nb * 4 * (3 if g3 else cw) / 2
                if acc > 80:
                    continue
                for rt in (16, 32):
                    lds = 2 * (_ceil(rt * M * cw, 256) + _ceil(rt * N * cw, 256)) * 256 * 4
                    if lds > LDS_BYTES:
                        continue
                    for il in (0, 1, 2):
                        if il and il + 1 > rt // 4:
                            continue
                        steps = rt // 4 if il == 0 else il + 1
                        ops = steps * (mb + nb) * cw / 2
                        for occ in (1, 2, 3, 4):
                            waves = occ * wpb
                            if waves % 4 or waves > 12 or occ * lds > LDS_BYTES:
                                continue
                            if acc + ops > (104 if waves <= 8 else 80):
                                continue
                            c = dict(kind="lds", MB=mb, NB=nb, WM=wm, WN=wn, RT=rt, WPB=wpb)
                            if occ > 1:
                                c["OCC"] = occ
                            if g3:
                                c["G3"] = 1
                            if il:
                                c["IL"] = il
                            out.append(c)
    return out


def _a32_candidates(op, dt, M, N):
    """Binary32-product kernels: the blocked matrix-core mappings with binary32
    operands.  Register model in binary64 units per lane: binary64 stretch
    sums (TSMTTSM) plus binary32 products (half a unit each) plus operands;
    kernels that still spill are dropped by the build."""
    cw = 2 if DTYPES[dt][1] else 1
    cplx = DTYPES[dt][1]
    out = []
    if op == "tsmttsm":
        if M <= 8 and N <= 8:
            return out
        mbt, nb = _ceil(M, 16), _ceil(N, 16)
        fl = max(f for f in (1, 2, 4) if (M * cw) % f == 0 and (N * cw) % f == 0)
        for mw in (1, 2, 4):
            if (mbt % mw and mw > 1) or mw > mbt:
                continue
            mb = _ceil(mbt, mw)
            acc = mb * nb * 4 * cw * 1.5
            for w in (4, 8):
                if w % mw:
                    continue
                for u in (1, 2, 4):
                    for nbuf in (2, 3):
                        ops = nbuf * u * (mb + nb) * cw / 2
                        if nbuf > 2 and u > 2:
                            continue
                        if acc + ops > (200 if w == 4 else 110):
                            continue
                        out.append(dict(kind="a32", MB=mb, NB=nb, MW=mw, U=u, WPB=w, NBUF=nbuf))
                        if mw == 1 and u <= 2:
                            out.append(dict(kind="a32", MB=mb, NB=nb, MW=mw, U=u, WPB=w, NBUF=nbuf, FL=fl))
                        # complex: three binary32 product sums per block (half a
                        # unit more than the two they replace)
                        if cplx and acc + mb * nb * 2 + ops <= (200 if w == 4 else 110):
                            out.append(dict(kind="a32", MB=mb, NB=nb, MW=mw, U=u, WPB=w, NBUF=nbuf, G3=1))
                            if mw == 1 and u <= 2:
                                out.append(dict(kind="a32", MB=mb, NB=nb, MW=mw, U=u, WPB=w, NBUF=nbuf, FL=fl,
                                                G3=1))
        return out + _lds32_candidates(op, dt, M, N)
    if M < 3 and N < 16:
        return out
    ms, nb = _ceil(M, 4), _ceil(N, 16)
    fl = max(f for f in (1, 2, 4) if M % f == 0)
    for u in (1, 2, 4):
        for w in (4, 8):
            for nbuf in (2, 3):
                ops = (nbuf * u * ms * cw + u * nb * 4 * cw) / 2
                if ops > (48 if w == 8 else 80) or (nbuf > 2 and u > 2):
                    continue
                out.append(dict(kind="a32", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf))
                if not cplx:
                    out.append(dict(kind="a32", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf, FL=fl))
                elif ops + u * nb * 2 <= (48 if w == 8 else 80):
                    out.append(dict(kind="a32", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf, G3=1))
    return out


def _mfma_blocks(mbt, nb, cplx, nbufs=(2, 3, 4), occ=True):
    """Matrix-core TSMTTSM configurations for a grid of mbt x nb 16 x 16
    blocks of C (shared by the exact-width and run-time-width variants)."""
    cw = 2 if cplx else 1
    out = []
    for mw in (1, 2, 3, 4):
        if (mbt % mw and mw > 1) or mw > mbt:
            continue
        mb = _ceil(mbt, mw)
        acc = mb * nb * 4 * cw
        # three m-slices (widths 33..48) need blocks of a multiple of three waves
        for w in ((6, 12) if mw == 3 else (4, 8)):
            # 256-thread blocks may use the whole register file of one
            # wave per SIMD: room for the 3 x 3 complex block grid
            # (widths 33..48), which no wave split divides
            if w % mw or acc > (72 if w == 4 else 64):
                continue
            for u in (1, 2, 4):
                for nbuf in nbufs:
                    ops = nbuf * u * (mb + nb) * cw
                    if ops > 72 or (nbuf > 2 and u > 2):
                        continue
                    # two waves per SIMD (OCC = 2, implied by 384- and
                    # 512-thread blocks) leave each lane 256 registers in
                    # all, three (768 threads) about 170
                    two = acc + ops <= 104
                    if (w > 4 and not two) or (w == 12 and acc + ops > 72):
                        continue
                    c = dict(kind="mfma", MB=mb, NB=nb, MW=mw, U=u, WPB=w, NBUF=nbuf)
                    out.append(c)
                    if occ and w == 4 and two and mw > 1:
                        out.append(dict(c, OCC=2))
                    # complex: Gauss's three-product form needs a third
                    # accumulator set (half the size of the two it replaces)
                    acc3 = mb * nb * 4 * 3
                    if cplx and acc3 <= 64 and (w == 4 or acc3 + ops <= 104):
                        out.append(dict(c, G3=1))
    return out


def _mfma_slices(ms, nb, cplx, va=False, nbufs=(2, 3, 4), cg=False):
    """Matrix-core TSMM configurations for a contraction depth of ms 4-wide
    slices and nb 16-column blocks of B (shared by the exact-width and
    run-time-width variants); ``va`` adds the paired loads of A, ``cg`` a
    twin of each plain one that reads its C operands from global memory at
    every tile instead of the LDS copy (an ablation of the C source)."""
    cw = 2 if cplx else 1
    out = []
    for u in (1, 2, 4):
        for w in (4, 8):
            for nbuf in nbufs:
                ops = nbuf * u * ms * cw + u * nb * 4 * cw
                if ops <= (96 if w == 8 else 160) and (nbuf == 2 or u <= 2):
                    if va:
                        out.append(dict(kind="mfma", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf, VA=1))
                    out.append(dict(kind="mfma", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf))
                    if cg:
                        out.append(dict(kind="mfma", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf, CG=1))
                    # complex three-product form: one more accumulator set, C staged three times
                    if cplx and ops + u * nb * 4 <= (96 if w == 8 else 160):
                        out.append(dict(kind="mfma", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf, G3=1))
    return out


def _slab_slices(ms, nb, M, es, fl):
    """TSMM configurations with slab reads of A (runs of 16 U rows of M
    elements of es bytes, loads of fl elements per lane), for a contraction
    depth of ms slices and nb column blocks; M is the widest run (for
    run-time widths: 4 ms)."""
    out = []
    for u in (1, 2, 4):
        for w in (4, 8):
            for nbuf in (2, 3):
                nl = _ceil(16 * u * M, 64 * fl) * fl * es // 8   # registers (doubles) per lane and tile
                ops = nbuf * nl + u * ms + u * nb * 4
                lds = w * 16 * u * M * es + ms * nb * 64 * 8
                if ops <= (96 if w == 8 else 160) and lds <= 64 * 1024 and (nbuf == 2 or u <= 2):
                    out.append(dict(kind="mfma", MS=ms, NB=nb, U=u, WPB=w, NBUF=nbuf, FL=fl))
    return out


def _candidates(op, dt, M, N):
    cw = 2 if DTYPES[dt][1] else 1
    cplx = DTYPES[dt][1]
    out = []
    # Register sets in flight (leap-frog ring depth): 2 = current + next.
    # 512-thread blocks cap a lane at 256 registers in all (VGPR + AGPR).
    if op == "tsmttsm":
        if M <= 16 and N <= 16:
            for u in (1, 2, 4, 8):
                for w in (4, 8):
                    for nbuf in (2, 4):
                        out.append(dict(kind="packed", U=u, WPB=w, NBUF=nbuf))
        if M == 1 and N == 1 and not cplx and not is_f32(dt):
            # the dot product: pairs of rows as 16-byte loads (contiguous vectors)
            for u in (1, 2, 4, 8):
                for w in (4, 8):
                    out.append(dict(kind="dot", U=u, WPB=w))
        if M * N * cw <= 64:
            for u in (1, 2, 4):
                if _valu_regs(op, M, N, cw, u) <= 110:
                    out.append(dict(kind="valu", MX=M, NX=N, U=u, VA=int(not cplx and M % 2 == 0),
                                    VB=int(not cplx and N % 2 == 0), WPB=WPB))
        if M > 8 or N > 8:
            out += _mfma_blocks(_ceil(M, 16), _ceil(N, 16), cplx)
        # tails on the vector unit: full blocks on the matrix cores, the
        # M mod 16 rows and N mod 16 columns of C as FMAs (one wave per row group)
        rm, rn = M % 16, N % 16
        if (rm or rn) and M > 16 and N > 16 and max(rm, rn) <= (4 if cplx else 8):
            mb, nb = _ceil(M, 16), _ceil(N, 16)
            mf, nf = mb - (1 if rm else 0), nb - (1 if rn else 0)
            tails = (mb * rn + nf * rm) * cw                 # doubles of tail sums per lane
            for g3 in ((0, 1) if cplx else (0,)):
                acct = mf * nf * 4 * (3 if g3 else cw)       # matrix-core accumulators
                for w in (4, 8):
                    for u in (1, 2, 4):
                        for nbuf in (2, 3):
                            ops = nbuf * u * (mb + nb) * cw
                            if ops > 72 or (nbuf > 2 and u > 2):
                                continue
                            if acct + ops + tails + u * cw <= (160 if w == 4 else 104):
                                out.append(dict(kind="mfma", MB=mb, NB=nb, MW=1, U=u, WPB=w, NBUF=nbuf, TL=1,
                                                **({"G3": 1} if g3 else {})))
        # slab reads of A and B (rows contiguous), with or without vector tails
        # (and, complex, with or without the three-product form)
        if M > 8 or N > 8:
            es = 4 if is_f32(dt) else 8                        # bytes per real storage element
            fl = max(f for f in (1, 2, 4) if (M * cw) % f == 0 and (N * cw) % f == 0 and f * es <= 16)
            mb, nb = _ceil(M, 16), _ceil(N, 16)
            rm, rn = M % 16, N % 16
            tails_ok = (rm or rn) and M > 16 and N > 16 and max(rm, rn) <= (4 if cplx else 8)
            for tl in ((0, 1) if tails_ok else (0,)):
                for g3 in ((0, 1) if cplx else (0,)):
                    mf, nf = (mb - (1 if rm else 0), nb - (1 if rn else 0)) if tl else (mb, nb)
                    acct = mf * nf * 4 * (3 if g3 else cw) + ((mb * rn + nf * rm) * cw if tl else 0)
                    if acct > 72:
                        continue
                    for w in (4, 8):
                        for u in (1, 2, 4):
                            for nbuf in (2, 3):
                                nl = (_ceil(4 * u * M * cw, 64 * fl) + _ceil(4 * u * N * cw, 64 * fl)) * fl * es // 8
                                ops = nbuf * nl + u * (mb + nb) * cw
                                lds = w * 4 * u * (M + N) * cw * es + M * N * cw * 8
                                # (wide block grids: one wave per SIMD and two register sets only)
                                if acct > 36 and (w > 4 or nbuf > 2):
                                    continue
                                if (acct + ops <= (160 if w == 4 else 104) and lds <= 64 * 1024
                                        and (nbuf == 2 or u <= 2)):
                                    c = dict(kind="mfma", MB=mb, NB=nb, MW=1, U=u, WPB=w, NBUF=nbuf, FL=fl)
                                    if tl:
                                        c["TL"] = 1
                                    if g3:
                                        c["G3"] = 1
                                    out.append(c)
        return out
    if M * cw <= 8 and N * cw <= 8:
        for u in (1, 2, 4):
            out.append(dict(kind="valu", MX=M, NX=N, U=u, VA=int(not cplx and M % 2 == 0),
                            VB=int(not cplx and N % 2 == 0), WPB=WPB))
    if N <= 16 and M <= 16 and _ceil((16 // N) * M, 4) <= 16:
        for u in (1, 2, 4):
            for w in (4, 8):
                for nbuf in (2, 4):
                    out.append(dict(kind="packed", U=u, WPB=w, NBUF=nbuf))
    # matrix cores from three columns of A up (one 4-deep slice with a zero
    # fourth column already beats row packing at 3 x 3; at 1 and 2 the
    # vector and packed kernels stay ahead)
    if M >= 3 or N >= 16:
        ms, nb = _ceil(M, 4), _ceil(N, 16)
        out += _mfma_slices(ms, nb, cplx, va=not cplx and M % 8 == 0, cg=True)
        # slab reads of A (rows contiguous): the wave's 16 U rows as one run of
        # loads of up to 16 bytes per lane, redistributed through LDS
        if not cplx:
            es = 4 if is_f32(dt) else 8                       # bytes per stored element
            fl = max(f for f in (1, 2, 4) if M % f == 0 and f * es <= 16)
            out += _slab_slices(ms, nb, M, es, fl)
    return out


def default_config(op, dt, M, N):
    """Heuristic configuration of one variant when the autotuner has not
    measured this (op, dt, M, N): row packing on the matrix cores for narrow
    widths, the blocked matrix-core kernels otherwise."""
    cw = 2 if DTYPES[dt][1] else 1
    if is_a32(dt):
        # binary32 products wherever the matrix-core mappings apply
        if op == "tsmttsm" and (M > 8 or N > 8):
            mbt, nb = _ceil(M, 16), _ceil(N, 16)
            mw = 1 if mbt * nb * cw <= 8 else 2
            return dict(kind="a32", MB=_ceil(mbt, mw), NB=nb, MW=mw, U=2, WPB=WPB)
        if op == "tsmm" and M >= 3:
            ms, nb = _ceil(M, 4), _ceil(N, 16)
            return dict(kind="a32", MS=ms, NB=nb, U=2 if ms * nb * cw <= 32 else 1, WPB=WPB)
        return default_config(op, A32_TWIN[dt], M, N)
    if op == "tsmttsm":
        if M <= 16 and N <= 16 and (M < 16 or N < 16):
            return dict(kind="packed", U=4, WPB=WPB)
        mbt, nb = _ceil(M, 16), _ceil(N, 16)
        mw = 1
        while mbt * nb * 4 * cw > 32 * mw and mw < mbt:
            mw *= 2
        mb = _ceil(mbt, mw)
        u = max(1, min(4, 8 // ((mb + nb) * cw)))
        return dict(kind="mfma", MB=mb, NB=nb, MW=mw, U=u, WPB=WPB)
    if M * cw <= 2 and N * cw <= 2 and not is_f32(dt):
        return dict(kind="valu", MX=M, NX=N, U=4, VA=int(cw == 1 and M % 2 == 0),
                    VB=int(cw == 1 and N % 2 == 0), WPB=WPB)
    if N <= 16 and M <= 16 and _ceil((16 // N) * M, 4) <= 16 and N < 16:
        return dict(kind="packed", U=2, WPB=WPB)
    ms, nb = _ceil(M, 4), _ceil(N, 16)
    u = 2 if (4 * ms * cw + 8 * nb * cw) <= 96 else 1
    return dict(kind="mfma", MS=ms, NB=nb, U=u, WPB=WPB)


# Run-time-width configurations chosen by a probe of non-square pairs at
# K = 2^24 (forced variants, median of three calls):
#   TSMTTSM block grid (m blocks, n blocks) -> (MB, NB, MW, U, WPB), real / complex.
#   The 2 x 3, 3 x 2 and 3 x 3 grids halve the time of pairs such as 17 x 33
#   (D 2.88 -> 1.35 ms, Z 7.7 -> 3.7 ms) that the 2 x 4 / 4 x 2 grids padded;
#   two rows in flight and eight waves took 30 x 60 from 3.16 to 2.05 ms (D).
_GEN_TSMTTSM = {
    (1, 2): ((1, 2, 1, 2, 4), (1, 2, 1, 1, 4)),
    (2, 1): ((2, 1, 1, 2, 4), (2, 1, 1, 1, 4)),
    (2, 2): ((2, 2, 1, 2, 8), (2, 2, 1, 2, 8)),
    (1, 4): ((1, 4, 1, 1, 4), (1, 4, 1, 1, 4)),
    (4, 1): ((4, 1, 1, 1, 4), (4, 1, 1, 1, 4)),
    (2, 3): ((2, 3, 1, 2, 8), (1, 3, 2, 2, 8)),
    (3, 2): ((3, 2, 1, 2, 8), (3, 2, 1, 2, 4)),
    (3, 3): ((3, 3, 1, 2, 8), (1, 3, 3, 1, 12)),
    (2, 4): ((2, 4, 1, 2, 8), (2, 4, 1, 1, 4)),
    (4, 2): ((4, 2, 1, 2, 8), (2, 2, 2, 2, 8)),
    (4, 4): ((2, 4, 2, 1, 4), (1, 4, 4, 1, 4)),
}
#   TSMM contraction depth in 4-wide slices and n blocks -> (U, WPB).
#   Depths of 6 and 12 slices (M <= 24, M <= 48) run 17 x 9 in 1.17 instead
#   of 1.40 ms and 40 x 8 in 2.19 instead of 2.79 ms (D).


def _gen_tsmm_cfg(ms, nb, cplx):
    if ms <= 2:
        return (2 if cplx or ms == 2 else 4), 8
    if ms in (6, 12):
        if not cplx:
            return 2, 8
        return (2 if ms == 6 and nb == 1 else 1), (4 if ms == 12 and nb == 4 else 8)
    cw = 2 if cplx else 1
    return (2 if (4 * ms * cw + 8 * nb * cw) <= 96 else 1), WPB


# Run-time-width classes, each listed before every class that contains it
# (the runtime takes the first record that covers (M, N), so a pair runs on
# its smallest covering class).  TSMTTSM: grids of (m, n) 16 x 16 blocks of
# C up to 4 x 4 (1 x 1 is row packing's); TSMM: contraction depths of ms
# 4-wide slices times n blocks of 16 columns of B.
GEN_TSMTTSM_CLASSES = sorted(((a, b) for a in range(1, 5) for b in range(1, 5) if (a, b) != (1, 1)),
                             key=lambda c: (c[0] * c[1], c))
GEN_TSMM_MS = (1, 2, 3, 4, 6, 8, 10, 12, 14, 16)
GEN_TSMM_CLASSES = sorted(((ms, nb) for ms in GEN_TSMM_MS for nb in range(1, 5)), key=lambda c: (c[0] * c[1], c))
GEN_TUNED_DTYPES = ("r64", "c128")


def generic_limits(op, cls):
    """(maxM, maxN) a run-time-width class serves."""
    return (16 * cls[0], 16 * cls[1]) if op == "tsmttsm" else (4 * cls[0], 16 * cls[1])


def generic_capacity(op, cfg):
    """(maxM, maxN) a matrix-core configuration can compute."""
    if op == "tsmttsm":
        return 16 * cfg["MB"] * cfg["MW"], 16 * cfg["NB"]
    return 4 * cfg["MS"], 16 * cfg["NB"]


def _next(values, x):
    later = [v for v in values if v > x]
    return later[0] if later else x


def generic_candidates(op, dt, cls):
    """Configurations the autotuner times for one run-time-width class: the
    matrix-core kernels of the class's own grid and of the grids one step
    larger in either dimension (padding a dimension can pay where a wider
    grid fits the waves better)."""
    cplx = DTYPES[dt][1]
    out, seen = [], set()
    if op == "tsmttsm":
        a, b = cls
        shapes = [(a, b), (_next((1, 2, 3, 4), a), b), (a, _next((1, 2, 3, 4), b))]
        for sh in shapes:
            for c in _mfma_blocks(sh[0], sh[1], cplx, nbufs=(2,), occ=False):
                key = json.dumps(c, sort_keys=True)
                if key not in seen:
                    seen.add(key)
                    out.append(c)
    else:
        ms, nb = cls
        shapes = [(ms, nb), (_next(GEN_TSMM_MS, ms), nb), (ms, _next((1, 2, 3, 4), nb))]
        for sh in shapes:
            cs = _mfma_slices(sh[0], sh[1], cplx, nbufs=(2, 3))
            if not cplx and not is_f32(dt):
                # slab reads of A with single-element loads (any M; rows contiguous)
                cs += _slab_slices(sh[0], sh[1], 4 * sh[0], 8, 1)
            for c in cs:
                key = json.dumps(c, sort_keys=True)
                if key not in seen:
                    seen.add(key)
                    out.append(c)
    return out


def generic_pairs(op, cls):
    """Pairs (M, N) a run-time-width class is timed on: in each dimension the
    smallest, middle and largest width the class serves as the tightest
    class (combined so that no pair is square: squares have kernels of their
    own)."""
    def spans(lo_step, values, x):
        prev = max([v for v in values if v < x], default=0)
        lo, hi = lo_step * prev + 1, lo_step * x
        return lo, (lo + hi) // 2, hi
    if op == "tsmttsm":
        m = spans(16, (1, 2, 3, 4), cls[0])
    else:
        m = spans(4, GEN_TSMM_MS, cls[0])
    n = spans(16, (1, 2, 3, 4), cls[1])
    pairs = [(m[0], n[1]), (m[1], n[2]), (m[2], n[0])]
    return [(M, N) if M != N else (M, N - 1 if N > 1 else N + 1) for M, N in pairs]


def tuned_generic(path=None):
    """{(op, dt, maxM, maxN): cfg} of the run-time-width classes chosen by the
    autotuner (tuned.json key "generic")."""
    path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            for e in json.load(f).get("generic", []):
                key = (e["op"], e["dt"], int(e["maxM"]), int(e["maxN"]))
                out[key] = e["cfg"]
                if e.get("plain_cfg"):
                    out[key + ("plain",)] = e["plain_cfg"]
    return out


def _tsmm_rb(cfg, cplx):
    """The twin of a TSMM run-time-width configuration that reads the old B
    with A (calls with beta != 0): the depth and blocks of the beta = 0
    kernel, rows in flight and waves by the register budget of the B ring."""
    u, w = _gen_tsmm_cfg(cfg["MS"], cfg["NB"], cplx)
    c = dict(kind="mfma", MS=cfg["MS"], NB=cfg["NB"], U=u, WPB=w, RB=1)
    if cfg["MS"] >= 6:
        c["WPB"] = WPB
    return c


def generic_variants(tuned_path=None):
    """Run-time-width variants: every (M, N) in [1, 64]^2 is served by one.
    The runtime takes the first one that covers (M, N), so each list runs
    from the smallest covering shape to the largest.  The binary64 types
    take the autotuned classes where the table has them."""
    tuned = tuned_generic(tuned_path)
    out = []
    for dt, (_, cplx) in DTYPES.items():
        if is_a32(dt):
            continue  # served by the run-time-width variants of the binary64-arithmetic twin
        # TSMTTSM: row packing up to 16, then blocked matrix-core kernels
        out.append(dict(op="tsmttsm", dt=dt, M=0, N=0, maxM=16, maxN=16,
                        cfg=dict(kind="packed", U=4, WPB=WPB)))
        auto = dt in GEN_TUNED_DTYPES and any(k[0] == "tsmttsm" and k[1] == dt for k in tuned)
        if auto:
            for cls in GEN_TSMTTSM_CLASSES:
                mx, nx = generic_limits("tsmttsm", cls)
                cfg = tuned.get(("tsmttsm", dt, mx, nx))
                if cfg:
                    out.append(dict(op="tsmttsm", dt=dt, M=0, N=0, maxM=mx, maxN=nx, cfg=cfg))
        for (mbt, nb), cfgs in _GEN_TSMTTSM.items():
            if auto and ("tsmttsm", dt, 16 * mbt, 16 * nb) in tuned:
                continue
            mb, nbb, mw, u, w = cfgs[1 if cplx else 0]
            out.append(dict(op="tsmttsm", dt=dt, M=0, N=0, maxM=16 * mbt, maxN=16 * nb,
                            cfg=dict(kind="mfma", MB=mb, NB=nbb, MW=mw, U=u, WPB=w)))
        # TSMM: the vector kernel only up to 2 x 2 (with run-time widths it
        # keeps C in registers sized for the maximum and falls far behind the
        # matrix cores beyond that: 0.3-1 TB/s at 1 x 8, 3 x 8, 1 x 4), then
        # matrix-core kernels whose contraction depth follows M in 4-wide
        # slices (one or two slices for M <= 8: 4.4-5.3 TB/s at 3 x 8, 1 x 8,
        # 8 x 3, where four slices reached 3-4 TB/s)
        if not is_f32(dt):
            out.append(dict(op="tsmm", dt=dt, M=0, N=0, maxM=2, maxN=2,
                            cfg=dict(kind="valu", MX=2, NX=2, U=2, VA=0, VB=0, WPB=WPB)))
        auto = dt in GEN_TUNED_DTYPES and any(k[0] == "tsmm" and k[1] == dt for k in tuned)
        if auto:
            tsmm = []
            for cls in GEN_TSMM_CLASSES:
                mx, nx = generic_limits("tsmm", cls)
                cfg = tuned.get(("tsmm", dt, mx, nx))
                if cfg:
                    tsmm.append((mx, nx, cfg))
                    # slab reads need contiguous rows: the fastest kernel
                    # without that need follows for other layouts
                    if needs_layout(cfg):
                        plain = tuned.get(("tsmm", dt, mx, nx, "plain"))
                        if not plain:
                            u, w = _gen_tsmm_cfg(cfg["MS"], cfg["NB"], cplx)
                            plain = dict(kind="mfma", MS=cfg["MS"], NB=cfg["NB"], U=u, WPB=w)
                        tsmm.append((mx, nx, plain))
        else:
            tsmm = []
            shapes = [(1, 1), (2, 1)] + [(ms, nb) for ms in (4, 6, 8, 12, 16) for nb in (1, 2, 4)]
            for ms, nb in shapes:
                u, w = _gen_tsmm_cfg(ms, nb, cplx)
                tsmm.append((4 * ms, 16 * nb, dict(kind="mfma", MS=ms, NB=nb, U=u, WPB=w)))
        done = set()
        for mx, nx, cfg in tsmm:
            # a twin reading the old B with A serves calls with beta != 0 (its
            # register ring of B does not fit eight-wave blocks from 6 slices)
            if (mx, nx) not in done:
                done.add((mx, nx))
                out.append(dict(op="tsmm", dt=dt, M=0, N=0, maxM=mx, maxN=nx, cfg=_tsmm_rb(cfg, cplx)))
            out.append(dict(op="tsmm", dt=dt, M=0, N=0, maxM=mx, maxN=nx, cfg=cfg))
    return out


def tuning_variants(widths):
    """All candidates of every (op, dtype, width) in ``widths``, plus the
    run-time-width variants (the library the autotuner times)."""
    out = []
    seen = set()
    for op in OPS:
        for dt in DTYPES:
            for (M, N) in widths:
                if is_f32(dt) and (M, N) not in PRECISION:
                    continue
                # binary32-arithmetic types: only their own kernels (the
                # binary64-arithmetic ones are timed under the twin type)
                cands = _a32_candidates(op, dt, M, N) if is_a32(dt) else candidates(op, dt, M, N)
                for c in cands:
                    v = dict(op=op, dt=dt, M=M, N=N, maxM=M, maxN=N, cfg=c)
                    name = variant_name(v)
                    if name not in seen:
                        seen.add(name)
                        out.append(v)
    return out + generic_variants()


def load_tuned(path):
    """{(op, dt, M, N): cfg} of the tuning table; an entry whose fastest
    configuration has access requirements (paired or slab reads of A) also
    names the fastest one without them, under the key (op, dt, M, N, "plain")."""
    out = {}
    if path and os.path.exists(path):
        with open(path) as f:
            tab = json.load(f)
        for e in tab.get("entries", []):
            key = (e["op"], e["dt"], int(e["M"]), int(e["N"]))
            out[key] = e["cfg"]
            if e.get("plain_cfg"):
                out[key + ("plain",)] = e["plain_cfg"]
    return out


def needs_layout(cfg):
    """True if a configuration reads A in a way only some layouts allow
    (paired loads, slab reads, direct loads of whole stages into LDS)."""
    return bool(cfg.get("VA") or cfg.get("FL") or cfg.get("kind") in ("lds", "dot"))


def exact_variants(widths, tuned=None):
    """One variant per (op, dtype, width); where the chosen one needs a layout
    of A (paired or slab reads), a second one without that need follows it,
    so calls with another leading dimension or alignment keep an exact-width
    kernel (the runtime takes the first record whose requirements hold)."""
    tuned = tuned or {}
    out = []
    for op in OPS:
        for dt in DTYPES:
            for (M, N) in widths:
                if is_f32(dt) and (M, N) not in PRECISION:
                    continue
                cfg = tuned.get((op, dt, M, N)) or default_config(op, dt, M, N)
                cfgs = [cfg]
                if needs_layout(cfg):
                    plain = tuned.get((op, dt, M, N, "plain")) or default_config(op, dt, M, N)
                    if not needs_layout(plain):
                        cfgs.append(plain)
                for c in cfgs:
                    # TSMM on the matrix cores: a twin reading the old B with A
                    # for calls with beta != 0, ahead of the one serving beta = 0
                    if op == "tsmm" and c["kind"] in ("mfma", "a32"):
                        out.append(dict(op=op, dt=dt, M=M, N=N, maxM=M, maxN=N, cfg=dict(c, RB=1)))
                    out.append(dict(op=op, dt=dt, M=M, N=N, maxM=M, maxN=N, cfg=c))
    return out


# ------------------------------------------------------------------ emission
def variant_name(v):
    c = v["cfg"]
    w = "%dx%d" % (v["M"], v["N"]) if v["M"] else "le%dx%d" % (v["maxM"], v["maxN"])
    if c["kind"] == "valu":
        tag = "valu_u%d" % c["U"]
    elif c["kind"] == "dot":
        tag = "dot_u%d" % c["U"]
    elif c["kind"] == "packed":
        tag = "packed_u%d" % c["U"]
    elif c["kind"] == "a32" and v["op"] == "tsmttsm":
        tag = "a32_b%dx%dw%d_u%d" % (c["MB"], c["NB"], c["MW"], c["U"])
    elif c["kind"] == "a32":
        tag = "a32_s%dn%d_u%d" % (c["MS"], c["NB"], c["U"])
    elif c["kind"] == "lds":
        tag = "lds_b%dx%dw%dx%d_k%d" % (c["MB"], c["NB"], c["WM"], c["WN"], c["RT"])
    elif v["op"] == "tsmttsm":
        tag = "mfma_b%dx%dw%d_u%d" % (c["MB"], c["NB"], c["MW"], c["U"])
    else:
        tag = "mfma_s%dn%d_u%d" % (c["MS"], c["NB"], c["U"])
    if c.get("WPB", WPB) != WPB:
        tag += "_w%d" % c["WPB"]
    if c.get("NBUF", 2) != 2:
        tag += "_r%d" % c["NBUF"]
    if c["kind"] == "mfma" and c.get("VA"):
        tag += "_v2"
    if c.get("OCC", 1) != 1:
        tag += "_o%d" % c["OCC"]
    if c.get("G3"):
        tag += "_g3"
    if c.get("FL"):
        tag += "_f%d" % c["FL"]
    if c.get("TL"):
        tag += "_t"
    if c.get("RB"):
        tag += "_rb"
    if c.get("CG"):
        tag += "_cg"
    if c.get("IL"):
        tag += "_il%d" % c["IL"]
    return "%s_%s_%s_%s" % (v["op"], v["dt"], w, tag)


def _template(v):
    c = v["cfg"]
    cplx = "true" if DTYPES[v["dt"]][1] else "false"
    M, N = v["M"], v["N"]
    nbuf = c.get("NBUF", 2)
    f32 = "true" if is_f32(v["dt"]) else "false"
    if c["kind"] == "packed":
        return "tsg::%s_packed<%d, %d, %d, %s, %d, %d, %s>" % (v["op"], M, N, c["U"], cplx, c["WPB"], nbuf, f32)
    if c["kind"] == "dot":
        return "tsg::tsmttsm_dot<%d, %d>" % (c["U"], c["WPB"])
    if c["kind"] == "a32" and v["op"] == "tsmttsm":
        return "tsg::tsmttsm_a32<%d, %d, %d, %d, %d, %d, %s, %d, %d, %d, %d, %s>" % (
            M, N, c["MB"], c["NB"], c["MW"], c["U"], cplx, c["WPB"], nbuf, c.get("OCC", 1), c.get("FL", 0),
            "true" if c.get("G3") else "false")
    if c["kind"] == "a32":
        return "tsg::tsmm_a32<%d, %d, %d, %d, %d, %s, %d, %d, %d, %s, %s>" % (
            M, N, c["MS"], c["NB"], c["U"], cplx, c["WPB"], nbuf, c.get("FL", 0), "true" if c.get("RB") else "false",
            "true" if c.get("G3") else "false")
    if c["kind"] == "lds":
        return "tsg::tsmttsm_lds%s<%d, %d, %d, %d, %d, %d, %d, %s, %s, %d, %d>" % (
            "_a32" if is_a32(v["dt"]) else "",
            M, N, c["MB"], c["NB"], c["WM"], c["WN"], c["RT"], cplx, "true" if c.get("G3") else "false",
            c.get("OCC", 1), c.get("IL", 0))
    if v["op"] == "tsmttsm":
        if c["kind"] == "valu":
            return "tsg::tsmttsm_valu<%d, %d, %d, %d, %d, %s, %s, %s, %d>" % (
                M, N, c["MX"], c["NX"], c["U"], cplx, "true" if c["VA"] else "false",
                "true" if c["VB"] else "false", c["WPB"])
        return "tsg::tsmttsm_mfma<%d, %d, %d, %d, %d, %d, %s, %d, %d, %d, %s, %s, %s, %d>" % (
            M, N, c["MB"], c["NB"], c["MW"], c["U"], cplx, c["WPB"], nbuf, c.get("OCC", 1), f32,
            "true" if c.get("G3") else "false", "true" if c.get("TL") else "false", c.get("FL", 0))
    if c["kind"] == "valu":
        return "tsg::tsmm_valu<%d, %d, %d, %d, %d, %s, %s, %s, %d>" % (
            M, N, c["MX"], c["NX"], c["U"], cplx, "true" if c["VA"] else "false",
            "true" if c["VB"] else "false", c["WPB"])
    return "tsg::tsmm_mfma<%d, %d, %d, %d, %d, %s, %d, %d, %s, %d, %s, %s, %d, %s, %s>" % (
        M, N, c["MS"], c["NB"], c["U"], cplx, c["WPB"], nbuf, "true" if c.get("VA") else "false",
        c.get("OCC", 1), f32, "true" if c.get("G3") else "false", c.get("FL", 0),
        "true" if c.get("RB") else "false", "true" if c.get("CG") else "false")


def rows_per_tile(v):
    """Rows one block consumes per grid-stride step (for packed kinds: per packed row P = 1)."""
    c = v["cfg"]
    if c["kind"] == "packed":
        return (4 if v["op"] == "tsmttsm" else 16) * c["U"] * c["WPB"]
    if c["kind"] == "lds":
        return c["RT"]
    if c["kind"] == "dot":
        return 2 * 64 * c["U"] * c["WPB"]
    if v["op"] == "tsmttsm":
        return 64 * c["U"] * c["WPB"] if c["kind"] == "valu" else 4 * c["U"] * (c["WPB"] // c["MW"])  # mfma, a32
    return 64 * c["U"] * c["WPB"] if c["kind"] == "valu" else 16 * c["U"] * c["WPB"]


def _launcher(v, fn):
    tmpl = _template(v)
    threads = 64 * v["cfg"]["WPB"]
    if v["op"] == "tsmttsm":
        args = "p.K, p.M, p.N, p.A, p.lda, p.X, p.ldx, static_cast<double*>(p.Y), p.ldy, p.ws, p.conj"
    else:
        args = ("p.K, p.M, p.N, p.A, p.lda, static_cast<const double*>(p.X), p.ldx, p.Y, p.ldy, "
                "p.alpha, p.beta, p.conj, p.opc")
    return ("void %s(const tsg::Launch& p)\n{\n"
            "    hipLaunchKernelGGL((%s), dim3(p.grid), dim3(%d), 0, p.stream, %s);\n}\n"
            "const void* %s() { return reinterpret_cast<const void*>(&%s); }\n"
            % (fn, tmpl, threads, args, fn.replace("launch_", "kernel_"), tmpl))


def _record(v, fn):
    c = v["cfg"]
    # slab reads need 16-byte alignment (and, with lda = M, an even width) where
    # one lane load spans two or more elements (a complex element is two reals)
    slab_pairs = c.get("FL", 0) // (2 if DTYPES[v["dt"]][1] else 1) >= 2
    pair_a = int(c["kind"] in ("valu", "mfma", "a32") and (bool(c.get("VA")) or slab_pairs))
    pair_x = int((c["kind"] == "valu" and bool(c.get("VB"))) or (v["op"] == "tsmttsm" and slab_pairs))
    even = int(v["M"] == 0 and (pair_a or pair_x))
    pack = 0 if c["kind"] != "packed" else (1 if v["op"] == "tsmttsm" else 2)
    flat_a = int(bool(c.get("FL")) or c["kind"] in ("lds", "dot"))
    read_b = int(bool(c.get("RB")))
    align16 = int(c["kind"] in ("lds", "dot"))
    return ('    {%d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, %d, "%s", &%s, &%s},\n'
            % (OPS[v["op"]], DTYPES[v["dt"]][0], v["M"], v["N"], v["maxM"], v["maxN"], pair_a, pair_x, even,
               64 * c["WPB"], rows_per_tile(v), pack, flat_a, read_b, align16, variant_name(v),
               fn.replace("launch_", "kernel_"), fn))


# batched orthogonalisation: input bytes per slab and queue interleave (0: every
# slab item before any update item), used until the autotuner has chosen
ORTH_DEFAULTS = {"item_bytes": 4 << 20, "lag": 0}


def tuned_batched(path):
    """The batched form's parameters chosen by the autotuner (tuned.json key
    "batched"), else ORTH_DEFAULTS."""
    out = dict(ORTH_DEFAULTS)
    if path and os.path.exists(path):
        with open(path) as f:
            b = json.load(f).get("batched") or {}
        out.update({k: int(b[k]) for k in ORTH_DEFAULTS if k in b})
    return out


def emit(outdir, variants, per_file=6, exclude=(), batched=None):
    """Write gen/tsg_gen_XX.hip (instantiations + launchers) and gen/tsg_table.hip.
    Returns the list of written source files.  Files are only rewritten when
    their text changes, so unchanged units need no recompilation.  Variants
    named in ``exclude`` are compiled but left out of the registry table;
    ``batched`` holds the batched form's tuned parameters."""
    batched = dict(ORTH_DEFAULTS, **(batched or {}))
    os.makedirs(outdir, exist_ok=True)
    files = []
    recs = []
    decls = []
    nfiles = max(1, math.ceil(len(variants) / per_file))
    for fi in range(nfiles):
        chunk = variants[fi * per_file:(fi + 1) * per_file]
        body = ['// generated by codegen.py -- do not edit\n#include "tsg_kernels.hpp"\n'
                '#include "tsg_registry.hpp"\n\nnamespace tsg_gen {\n']
        for k, v in enumerate(chunk):
            fn = "launch_%s" % variant_name(v)
            body.append(_launcher(v, fn))
            decls.append("void %s(const tsg::Launch& p);\nconst void* %s();\n" % (fn, fn.replace("launch_", "kernel_")))
            if variant_name(v) not in exclude:
                recs.append((v, fn))
        body.append("}  // namespace tsg_gen\n")
        text = "".join(body)
        path = os.path.join(outdir, "tsg_gen_%02d.hip" % fi)
        _write_if_changed(path, text)
        files.append(path)
    table = ['// generated by codegen.py -- do not edit\n#include "tsg_registry.hpp"\n\nnamespace tsg_gen {\n']
    table.extend(decls)
    table.append("}  // namespace tsg_gen\n\n// host-only object: keep it out of the device compilation pass\n"
                 "#ifndef __HIP_DEVICE_COMPILE__\nnamespace tsg {\nusing namespace tsg_gen;\n"
                 "const Variant kVariants[] = {\n")
    for v, fn in recs:
        table.append(_record(v, fn))
    table.append("};\nconst int kNumVariants = %d;\n"
                 "// batched orthogonalisation (autotuned): input bytes per slab, queue interleave\n"
                 "const int64_t kOrthItemBytes = %d;\nconst int kOrthLag = %d;\n"
                 "}  // namespace tsg\n#endif\n" % (len(recs), batched["item_bytes"], batched["lag"]))
    path = os.path.join(outdir, "tsg_table.hip")
    _write_if_changed(path, "".join(table))
    files.append(path)
    # remove stale units from an earlier, larger variant set
    for f in os.listdir(outdir):
        p = os.path.join(outdir, f)
        if f.startswith("tsg_gen_") and p not in files:
            os.remove(p)
    return files


def _write_if_changed(path, text):
    if os.path.exists(path):
        with open(path) as f:
            if f.read() == text:
                return
    with open(path, "w") as f:
        f.write(text)


def all_variants(widths=None, tuned_path=None):
    widths = (GRADED + SQUARE_ALL + NARROW) if widths is None else widths
    seen = set()
    uniq = []
    for (M, N) in widths:
        if (M, N) not in seen:
            seen.add((M, N))
            uniq.append((M, N))
    return exact_variants(uniq, load_tuned(tuned_path)) + generic_variants(tuned_path)


def template_of(v):
    """C++ name of the kernel template instantiation of variant ``v``."""
    return _template(v)


def kernel_symbol(name, tuned=None):
    """Demangled symbol prefix ("void tsg::...<...>") of the product variant
    called ``name``, as profilers print it; None if no such variant."""
    tuned = tuned or os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
    for v in all_variants(None, tuned):
        if variant_name(v) == name:
            return "void " + _template(v)
    return None
