"""GPU parity of the batched block orthogonalisation (one persistent launch).

For every instance: C = V^T W (old W), then W_new = W - V C.  The check is
split so that each half has a tight bound of its own:
  * C against the compensated oracle, entry by entry within
    1e-12 * (|V|^T |W|) and normwise within 1e-12 ||C_ref||;
  * W_new against the oracle's update computed from the GPU's own C, entry
    by entry within 1e-12 * (|W| + |V| |C|).
Integer-valued inputs make both products exact in binary64: then C and
W_new must equal the oracle bit for bit.  With an orthonormal V (QR), the
projection leaves ||V^T W_new||_F <= 1e-13 ||W||_F.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1905_03136_amd import _lib, api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-12


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def check_bound(got, ref, bound, tol=TOL, what=""):
    err = np.abs(got - ref)
    assert np.all(err <= tol * bound + 1e-300), "%s: max elementwise excess %g" % (what, np.max(err - tol * bound))


def check_instance(V, W0, C_gpu, W_gpu, what=""):
    C_ref = oracle.tsmttsm(V, W0, compensated=True)
    check_bound(C_gpu, C_ref, np.abs(V).T @ np.abs(W0), what=what + " C")
    assert np.linalg.norm(C_gpu - C_ref) <= TOL * max(np.linalg.norm(C_ref), 1e-300), what
    W_ref = oracle.tsmm(V, C_gpu, W0.copy(), alpha=-1.0, beta=1.0, compensated=True)
    check_bound(W_gpu, W_ref, np.abs(W0) + np.abs(V) @ np.abs(C_gpu), what=what + " W")


# (K, M, N): the workload's widths, odd widths, a K smaller than a step, K = 1 and K = 0,
# and narrow widths whose first phase packs P = 16 / max(M, N) = 3, 2, 8, 5 rows per product
SHAPES = [(100003, 64, 16), (70001, 32, 8), (50000, 16, 4), (65536, 8, 1), (30011, 4, 16),
          (20001, 13, 7), (9999, 17, 16), (12345, 63, 15), (777, 3, 5), (15, 64, 1), (1, 1, 1),
          (0, 8, 4), (40000, 48, 12), (25000, 1, 16), (33333, 20, 3), (11111, 36, 11),
          (40009, 5, 3), (12007, 7, 2), (5003, 2, 1), (3001, 1, 3)]


def _instances(shapes, seed, integer=False):
    out = []
    for i, (K, M, N) in enumerate(shapes):
        if integer:
            V = inputs.host_integers(K, M, seed, inputs.STREAM_A + 2 * i, False, -7, 8)
            W = inputs.host_integers(K, N, seed, inputs.STREAM_B + 2 * i, False, -7, 8)
        else:
            V = inputs.host_uniform(K, M, seed, inputs.STREAM_A + 2 * i)
            W = inputs.host_uniform(K, N, seed, inputs.STREAM_B + 2 * i)
        out.append((V, W))
    return out


@pytest.mark.parametrize("rows_per_item", [0, 1000, 16, 4099])
def test_orth_batched_parity(rows_per_item):
    print("orth parity rows_per_item=%d" % rows_per_item, flush=True)
    host_inst = _instances(SHAPES, 31)
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    C = api.orth_batched(pairs, rows_per_item=rows_per_item)
    for i, ((V, W0), (dV, dW), dC) in enumerate(zip(host_inst, pairs, C)):
        check_instance(V, W0, host(dC), host(dW), "instance %d %s" % (i, SHAPES[i]))
        assert np.array_equal(host(dV), V)          # V is read only


def test_orth_batched_integer_exact():
    print("orth integer exact", flush=True)
    host_inst = _instances(SHAPES, 32, integer=True)
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    C = api.orth_batched(pairs, rows_per_item=2000)
    for i, ((V, W0), (_, dW), dC) in enumerate(zip(host_inst, pairs, C)):
        C_ref, W_ref = oracle.orth_step(V, W0)
        assert np.array_equal(host(dC), C_ref), "instance %d" % i
        assert np.array_equal(host(dW), W_ref), "instance %d" % i


def test_orth_batched_strided():
    """Leading dimensions larger than the widths (column slices of wider arrays)."""
    print("orth strided", flush=True)
    K = 54321
    Vfull = inputs.host_uniform(K, 40, 33, inputs.STREAM_A)
    Wfull = inputs.host_uniform(K, 24, 33, inputs.STREAM_B)
    dV, dW = dev(Vfull), dev(Wfull)
    Cbig = torch.full((30, 20), 7.0, dtype=torch.float64, device=DEV)
    plan = api.OrthPlan([(dV[:, 3:33], dW[:, 2:13])], rows_per_item=3000, C=[Cbig[:, 5:16]])
    plan.launch()
    plan.check()
    plan.close()
    V, W0 = Vfull[:, 3:33], Wfull[:, 2:13]
    check_instance(np.ascontiguousarray(V), np.ascontiguousarray(W0), host(Cbig[:, 5:16]),
                   host(dW[:, 2:13]), "strided")
    Wn = host(dW)
    assert np.array_equal(Wn[:, :2], Wfull[:, :2]) and np.array_equal(Wn[:, 13:], Wfull[:, 13:])
    Cb = host(Cbig)
    assert np.all(Cb[:, :5] == 7.0) and np.all(Cb[:, 16:] == 7.0)


# strided instances (leading dimensions above the widths) of every width class
# of the strided paths: updates in 1..16 four-column slices, partial sums in
# 1..4 sixteen-column blocks
STRIDED_M = [3, 4, 6, 11, 16, 19, 24, 27, 30, 36, 40, 44, 48, 52, 56, 60, 64]


@pytest.mark.parametrize("rows_per_item", [0, 1200])
def test_orth_batched_strided_every_width_class(rows_per_item):
    print("orth strided width classes rows_per_item=%d" % rows_per_item, flush=True)
    pairs, ref = [], []
    for i, M in enumerate(STRIDED_M):
        K, N = 3001 + 977 * i, 1 + (5 * i) % 16
        V = inputs.host_integers(K, M + 3, 40, inputs.STREAM_A + 2 * i, False, -7, 8)
        W = inputs.host_integers(K, N + 2, 40, inputs.STREAM_B + 2 * i, False, -7, 8)
        dV, dW = dev(V), dev(W)
        pairs.append((dV[:, 1:1 + M], dW[:, 2:2 + N]))
        ref.append((np.ascontiguousarray(V[:, 1:1 + M]), np.ascontiguousarray(W[:, 2:2 + N]), dW, W))
    C = api.orth_batched(pairs, rows_per_item=rows_per_item)
    for i, ((V, W0, dW, Wfull), dC) in enumerate(zip(ref, C)):
        C_ref, W_ref = oracle.orth_step(V, W0)
        assert np.array_equal(host(dC), C_ref), "instance %d M=%d C" % (i, STRIDED_M[i])
        Wn = host(dW)
        N = W0.shape[1]
        assert np.array_equal(Wn[:, 2:2 + N], W_ref), "instance %d M=%d W" % (i, STRIDED_M[i])
        # the columns around the instance's W are untouched
        assert np.array_equal(Wn[:, :2], Wfull[:, :2]) and np.array_equal(Wn[:, 2 + N:], Wfull[:, 2 + N:])


def test_orth_batched_orthogonality():
    print("orth orthogonality", flush=True)
    shapes = [(131072, 64, 16), (100000, 32, 8), (65536, 16, 4), (80000, 8, 1), (70000, 4, 16)]
    host_inst = []
    for i, (K, M, N) in enumerate(shapes):
        V = inputs.orthonormal_block(K, M, seed=34, stream=inputs.STREAM_V0 + i)
        W = inputs.host_uniform(K, N, 34, inputs.STREAM_B + i)
        host_inst.append((V, W))
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    api.orth_batched(pairs)
    for (V, W0), (_, dW) in zip(host_inst, pairs):
        Wn = host(dW)
        res = np.linalg.norm(V.T @ Wn) / np.linalg.norm(W0)
        assert res <= 1e-13, res


def test_orth_graph_replay_equals_direct_launch():
    """Replays of the captured graph give the direct launch's result bit for
    bit, with eager work (restoring W) and synchronisations in between."""
    print("orth graph replay", flush=True)
    host_inst = _instances(SHAPES[:8], 35)
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    W0 = [w.clone() for _, w in pairs]
    plan = api.OrthPlan(pairs, rows_per_item=5000)
    try:
        plan.run()
        plan.check()
        ref_C = [c.clone() for c in plan.C]
        ref_W = [w.clone() for _, w in pairs]
        for rep in range(4):
            for (_, w), w0 in zip(pairs, W0):
                w.copy_(w0)
            for c in plan.C:
                c.fill_(float("nan"))
            torch.cuda.synchronize()
            plan.launch()
            plan.check()
            for i in range(len(pairs)):
                assert torch.equal(plan.C[i], ref_C[i]), "replay %d instance %d" % (rep, i)
                assert torch.equal(pairs[i][1], ref_W[i]), "replay %d instance %d" % (rep, i)
    finally:
        plan.close()
    for i, ((V, w0), dC, dW) in enumerate(zip(host_inst, ref_C, ref_W)):
        check_instance(V, w0, host(dC), host(dW), "instance %d" % i)


def test_orth_on_side_stream():
    print("orth side stream", flush=True)
    host_inst = _instances(SHAPES[:6], 36)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pairs = [(dev(V), dev(W)) for V, W in host_inst]
        plan = api.OrthPlan(pairs)
        plan.launch()
    s.synchronize()
    plan.check()
    plan.close()
    for i, ((V, W0), (_, dW), dC) in enumerate(zip(host_inst, pairs, plan.C)):
        check_instance(V, W0, host(dC), host(dW), "instance %d" % i)


def test_orth_spin_limit_error_path():
    """A spin limit of 0 makes every update give up at once: the launch ends
    normally, check() reports the error, and the plan works again afterwards."""
    print("orth spin limit", flush=True)
    host_inst = _instances(SHAPES[:4], 37)
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    W0 = [w.clone() for _, w in pairs]
    plan = api.OrthPlan(pairs)
    try:
        plan.set_spin_limit(0)
        plan.launch()
        with pytest.raises(_lib.TsgError) as e:
            plan.check()
        assert e.value.status == _lib.TSG_E_HIP
        plan.check()                                 # the flag was cleared
        plan.set_spin_limit(1 << 23)
        for (_, w), w0 in zip(pairs, W0):
            w.copy_(w0)
        plan.launch()
        plan.check()
    finally:
        plan.close()
    for i, ((V, W0h), (_, dW), dC) in enumerate(zip(host_inst, pairs, plan.C)):
        check_instance(V, W0h, host(dC), host(dW), "instance %d" % i)


@pytest.mark.slow
def test_orth_full_size_sampled():
    """The 64-instance workload at full size (K_i log-uniform in [2^16, 2^22])
    in the launch configuration of the benchmark, checked on sampled entries
    of C_i and sampled rows of W_i for a few instances."""
    print("orth full size", flush=True)
    shapes = inputs.batched_instances(64, seed=0)
    pairs = []
    for i, (K, M, N) in enumerate(shapes):
        V = inputs.device_uniform(K, M, 40 + i, inputs.STREAM_A, False, DEV)
        W = inputs.device_uniform(K, N, 40 + i, inputs.STREAM_B, False, DEV)
        pairs.append((V, W))
    order = sorted(range(64), key=lambda i: shapes[i][0] * (shapes[i][1] + shapes[i][2]))
    pick = [order[-1], order[0], order[32]]
    W0 = {i: host(pairs[i][1]) for i in pick}
    plan = api.OrthPlan(pairs)
    plan.launch()
    plan.check()
    rng = np.random.default_rng(41)
    for i in pick:
        K, M, N = shapes[i]
        V = host(pairs[i][0])
        C = host(plan.C[i])
        ent = [(int(rng.integers(M)), int(rng.integers(N))) for _ in range(6)]
        ref = oracle.tsmttsm_entries(V, W0[i], ent)
        for (m, n), r in zip(ent, ref):
            bound = np.abs(V[:, m]) @ np.abs(W0[i][:, n])
            assert abs(C[m, n] - r) <= TOL * bound, (i, m, n)
        rows = np.sort(rng.choice(K, 64, replace=False))
        rows[-1] = K - 1
        Wn = host(pairs[i][1])[rows]
        ref_rows = oracle.tsmm_rows(V[rows], C, W0[i][rows], alpha=-1.0, beta=1.0)
        check_bound(Wn, ref_rows, np.abs(W0[i][rows]) + np.abs(V[rows]) @ np.abs(C), what="rows %d" % i)
    plan.close()


# ------------------------------------------------ descriptors in device memory
def test_orth_batched_device_descriptors_match_plan():
    """tsg_orth_batched (descriptors in device memory, queue built by the
    set-up kernel on every call) gives the plan's results bit for bit (same
    slabs, same summation orders) and meets the oracle's bounds; a second
    call on the same workspace does too."""
    print("orth device descriptors", flush=True)
    host_inst = _instances(SHAPES, 38)
    pairs_a = [(dev(V), dev(W)) for V, W in host_inst]
    pairs_b = [(dev(V), dev(W)) for V, W in host_inst]
    plan = api.OrthPlan(pairs_a)
    try:
        plan.launch()
        plan.check()
    finally:
        plan.close()
    batch = api.OrthBatch(pairs_b)
    batch.run()
    batch.check()
    for i in range(len(host_inst)):
        assert torch.equal(batch.C[i], plan.C[i]), "instance %d: C differs from the plan's" % i
        assert torch.equal(pairs_b[i][1], pairs_a[i][1]), "instance %d: W differs from the plan's" % i
    for i, ((V, W0), (_, dW), dC) in enumerate(zip(host_inst, pairs_b, batch.C)):
        check_instance(V, W0, host(dC), host(dW), "instance %d" % i)
    # again on the same workspace, from the original W
    for (_, w), (_, w0) in zip(pairs_b, host_inst):
        w.copy_(dev(w0))
    batch.run()
    batch.check()
    for i in range(len(host_inst)):
        assert torch.equal(batch.C[i], plan.C[i]) and torch.equal(pairs_b[i][1], pairs_a[i][1]), i


def test_orth_batched_integer_exact_device_descriptors():
    print("orth device descriptors integer", flush=True)
    host_inst = _instances(SHAPES, 39, integer=True)
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    batch = api.OrthBatch(pairs)
    batch.run()
    batch.check()
    for i, ((V, W0), (_, dW), dC) in enumerate(zip(host_inst, pairs, batch.C)):
        C_ref = oracle.tsmttsm(V, W0)
        assert np.array_equal(host(dC), C_ref), i
        assert np.array_equal(host(dW), oracle.tsmm(V, C_ref, W0.copy(), alpha=-1.0, beta=1.0)), i


def test_orth_batched_captured_graph_replays():
    """The call captured by the caller into a graph: every replay (with eager
    work restoring W and synchronisations between) equals the eager call bit
    for bit."""
    print("orth device descriptors graph", flush=True)
    host_inst = _instances(SHAPES[:10], 40)
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    W0 = [w.clone() for _, w in pairs]
    batch = api.OrthBatch(pairs)
    batch.run()
    batch.check()
    ref_C = [c.clone() for c in batch.C]
    ref_W = [w.clone() for _, w in pairs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            batch.run()
    torch.cuda.synchronize()
    for rep in range(4):
        for (_, w), w0 in zip(pairs, W0):
            w.copy_(w0)
        for c in batch.C:
            c.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        batch.check()
        for i in range(len(pairs)):
            assert torch.equal(batch.C[i], ref_C[i]), "replay %d instance %d" % (rep, i)
            assert torch.equal(pairs[i][1], ref_W[i]), "replay %d instance %d" % (rep, i)
    for i, ((V, w0), dC, dW) in enumerate(zip(host_inst, ref_C, ref_W)):
        check_instance(V, w0, host(dC), host(dW), "instance %d" % i)


def test_orth_batched_device_side_rejections():
    """Errors the host cannot see (the descriptors are in device memory) are
    found by the set-up kernel: nothing runs, every C and W is left as it
    was, and the check reports the cause; the next valid call works."""
    print("orth device descriptors rejections", flush=True)
    host_inst = _instances(SHAPES[:4], 41)
    pairs = [(dev(V), dev(W)) for V, W in host_inst]
    batch = api.OrthBatch(pairs)
    W0 = [w.clone() for _, w in pairs]
    for c in batch.C:
        c.fill_(7.0)
    # an invalid width written into the device copy of descriptor 2 (M = 65)
    good = batch.d_descs.clone()
    desc_size = batch.d_descs.numel() // len(pairs)
    bad = host(batch.d_descs).copy()
    bad[2 * desc_size + 8:2 * desc_size + 12] = np.frombuffer(np.int32(65).tobytes(), dtype=np.uint8)
    batch.d_descs.copy_(dev(bad))
    batch.run()
    with pytest.raises(_lib.TsgError) as e:
        batch.check()
    assert e.value.status == _lib.TSG_E_ARG
    for (_, w), w0, c in zip(pairs, W0, batch.C):
        assert torch.equal(w, w0) and bool(torch.all(c == 7.0))
    batch.check()                                           # the report was cleared
    # a workspace too small for the partial sums (but large enough for the queue)
    batch.d_descs.copy_(good)
    full = batch.workspace
    small = _lib.tsg_workspace_size(_lib.TSG_KIND_ORTH, _lib.TSG_R64, 1, 1, 1, len(pairs))  # queue, no room
    batch.workspace = full[:small]
    batch.run()
    with pytest.raises(_lib.TsgError) as e:
        batch.check()
    assert e.value.status == _lib.TSG_E_NOMEM
    for (_, w), w0 in zip(pairs, W0):
        assert torch.equal(w, w0)
    batch.workspace = full
    batch.run()
    batch.check()
    for i, ((V, W0h), (_, dW), dC) in enumerate(zip(host_inst, pairs, batch.C)):
        check_instance(V, W0h, host(dC), host(dW), "instance %d" % i)
