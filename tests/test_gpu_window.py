"""Sliding-window maintenance on the GPU (gsl_voxel_keys, gsl_window_classify,
gsl_window_compact) against the oracle's voxel key, classification and
swap-with-rear compaction (Sec. II-A eq. HashKey, Sec. II-C Steps 1-4).
Everything here is integer or data movement: bit-exact."""
import numpy as np
import pytest
import torch

import scenegen as S

from gpuutil import context, ops

pytestmark = pytest.mark.gpu

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
R_ROWS = 42


def _u64(t):
    return t.detach().cpu().numpy().view(np.uint64)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.uint64)).view(np.int64).copy()).cuda()


def _okeys(oracle, pts, vs):
    k, ok = oracle.voxel_key(pts, vs)
    k = k.copy()
    k[~ok] = EMPTY
    return k


def _odd_points(seed, P, vs):
    """Points on and next to voxel faces, negative, non-finite and out of range."""
    rng = np.random.default_rng(seed)
    p = rng.normal(scale=30.0, size=(P, 3)).astype(np.float32)
    q = P // 5
    p[:q] = (np.round(p[:q] / np.float32(vs)) * np.float32(vs)).astype(np.float32)  # on faces
    p[q:2 * q] = np.nextafter(p[:q], np.float32(-np.inf))  # just below them
    p[2 * q, 0] = np.nan
    p[2 * q + 1, 1] = np.inf
    p[2 * q + 2, 2] = -np.inf
    p[2 * q + 3, 0] = np.float32(vs) * np.float32(2 ** 20) * 1.01  # index beyond 2^20
    p[2 * q + 4, 1] = -np.float32(vs) * np.float32(2 ** 20)  # exactly -2^20: valid
    p[2 * q + 5, 2] = -np.float32(vs) * np.float32(2 ** 20) * 1.01
    return p


@pytest.mark.parametrize("vs", [0.5, 0.06, 1.0])
def test_voxel_keys_match_oracle(oracle, vs):
    O = ops()
    ctx = context()
    pts = _odd_points(11, 9000, vs)
    want = _okeys(oracle, pts, vs)
    aos = O.voxel_keys(ctx, torch.from_numpy(pts).cuda(), vs)
    soa = O.voxel_keys(ctx, torch.from_numpy(np.ascontiguousarray(pts.T)).cuda(), vs, component_major=True)
    torch.cuda.synchronize()
    assert np.array_equal(_u64(aos), want)
    assert np.array_equal(_u64(soa), want)
    assert (want == EMPTY).sum() == 5


def _classify(O, ctx, oracle, win_keys, pts, vs, n=None):
    """GPU and oracle classification; asserts they agree, returns the
    GPU's (D, A, add keys, workspace) and the oracle's delete flags."""
    n = len(win_keys) if n is None else n
    keys_d = _dev(win_keys)
    ws = O.window_workspace(ctx, n, len(pts))
    counts, add = O.window_classify(ctx, torch.from_numpy(pts).cuda(), vs, keys_d, n, ws)
    torch.cuda.synchronize()
    D, A = (int(x) for x in counts.cpu())
    pk, pok = oracle.voxel_key(pts, vs)
    d_want, add_want = oracle.window_classify(win_keys[:n], pk, pok)
    assert D == int(d_want.sum())
    assert A == len(add_want)
    assert np.array_equal(_u64(add[:A]), add_want)
    fov = pk[pok]
    return D, A, ws, fov, add_want


def _rows(seed, R, n):
    return np.random.default_rng(seed).normal(size=(R, n)).astype(np.float32)


@pytest.mark.parametrize("n,P", [(1, 1), (3000, 2000), (10_001, 9_003), (70_000, 20_000)])
def test_classify_matches_oracle(oracle, n, P):
    """D, A and the ADD keys in first-point order, for windows spanning
    several scan blocks with a ragged tail."""
    O = ops()
    ctx = context()
    frames, means = S.lidar_stream(21 + n, 2, P, n, extent=40.0, n_planes=150, range_m=12.0, step=1.5)
    vs = 0.5
    win = _okeys(oracle, means, vs)
    _classify(O, ctx, oracle, win, frames[1], vs)


def _step_both(O, ctx, oracle, keys_d, block_d, n, win_keys, win_rows, pts, vs, seed, per_voxel=2):
    """One frame on both sides; returns the oracle's new window."""
    D, A, ws, fov, add_vox = _classify(O, ctx, oracle, win_keys, pts, vs, n)
    rng = np.random.default_rng(seed)
    add_keys = np.repeat(add_vox, per_voxel)
    add_rows = rng.normal(size=(R_ROWS, len(add_keys))).astype(np.float32)
    ek, er, status = O.window_compact(ctx, keys_d, block_d, n, D, _dev(add_keys), torch.from_numpy(add_rows).cuda(),
                                      ws)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    k_w, r_w, ek_w, er_w = oracle.window_maintain(win_keys, win_rows, fov, add_keys, add_rows)
    n2 = len(k_w)
    assert n2 == n - D + len(add_keys)
    assert np.array_equal(_u64(keys_d[:n2]), k_w)
    assert np.array_equal(block_d[:, :n2].cpu().numpy().view(np.uint32), r_w.view(np.uint32))
    assert np.array_equal(_u64(ek), ek_w)
    assert np.array_equal(er.cpu().numpy().view(np.uint32), er_w.view(np.uint32))
    return k_w, r_w


@pytest.mark.parametrize("n,P,cap", [(5000, 4000, 9000), (40_000, 30_000, 60_000)])
def test_window_stream_matches_oracle(oracle, n, P, cap):
    """Four frames of a moving LiDAR: after each, the window (keys and all
    42 rows, bit for bit), the evicted Gaussians, and the counts agree."""
    O = ops()
    ctx = context()
    vs = 0.5
    frames, means = S.lidar_stream(31, 5, P, n, extent=50.0, n_planes=200, range_m=12.0, step=1.0)
    win_keys = _okeys(oracle, means, vs)
    win_rows = _rows(5, R_ROWS, n)
    keys_d = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
    keys_d[:n] = O.voxel_keys(ctx, torch.from_numpy(means).cuda(), vs)
    torch.cuda.synchronize()
    assert np.array_equal(_u64(keys_d[:n]), win_keys)
    block_d = torch.zeros(R_ROWS, cap, dtype=torch.float32, device="cuda")
    block_d[:, :n] = torch.from_numpy(win_rows).cuda()
    for f in range(1, 5):
        win_keys, win_rows = _step_both(O, ctx, oracle, keys_d, block_d, len(win_keys), win_keys, win_rows,
                                        frames[f], vs, seed=100 + f)


def test_window_edge_cases(oracle):
    """Empty window, empty frame, a frame of NaN returns only, no deletion,
    and every Gaussian deleted with new ones appended."""
    O = ops()
    ctx = context()
    vs = 0.5
    cap = 4000
    frames, means = S.lidar_stream(41, 2, 1500, 1200, extent=30.0, n_planes=80, range_m=10.0, step=1.0)

    def fresh(n_keys, rows):
        keys_d = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
        block_d = torch.zeros(R_ROWS, cap, dtype=torch.float32, device="cuda")
        if len(n_keys):
            keys_d[:len(n_keys)] = _dev(n_keys)
            block_d[:, :len(n_keys)] = torch.from_numpy(rows).cuda()
        return keys_d, block_d

    win = _okeys(oracle, means, vs)
    rows = _rows(6, R_ROWS, len(win))
    # empty window: every key of the frame is ADD
    k, b = fresh(np.zeros(0, np.uint64), None)
    _step_both(O, ctx, oracle, k, b, 0, np.zeros(0, np.uint64), np.zeros((R_ROWS, 0), np.float32), frames[0], vs, 1)
    # empty frame: everything is deleted
    k, b = fresh(win, rows)
    _step_both(O, ctx, oracle, k, b, len(win), win, rows, np.zeros((0, 3), np.float32), vs, 2)
    # NaN returns only
    k, b = fresh(win, rows)
    nanf = np.full((700, 3), np.nan, np.float32)
    _step_both(O, ctx, oracle, k, b, len(win), win, rows, nanf, vs, 3)
    # the frame's points are the window's means: no deletion, nothing to add
    k, b = fresh(win, rows)
    D, A, _, _, _ = _classify(O, ctx, oracle, win, means, vs)
    assert D == 0 and A == 0
    _step_both(O, ctx, oracle, k, b, len(win), win, rows, means, vs, 4)
    # far away frame: all deleted, all of the frame added
    k, b = fresh(win, rows)
    far = (frames[1] + np.float32(500.0)).astype(np.float32)
    _step_both(O, ctx, oracle, k, b, len(win), win, rows, far, vs, 5)
    # a single Gaussian that stays, a single point
    k, b = fresh(win[:1], rows[:, :1])
    _step_both(O, ctx, oracle, k, b, 1, win[:1], rows[:, :1], means[:1], vs, 6)


def test_window_compact_rejects_stale_counts(oracle):
    """A D that differs from the classification leaves the window untouched
    and sets the status word; sizes beyond the capacity fail on the host."""
    O = ops()
    A_ = O.A
    ctx = context()
    vs = 0.5
    frames, means = S.lidar_stream(51, 2, 3000, 2500, extent=30.0, n_planes=80, range_m=10.0, step=1.0)
    win = _okeys(oracle, means, vs)
    n, cap = len(win), 2600
    keys_d = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
    keys_d[:n] = _dev(win)
    block_d = torch.zeros(R_ROWS, cap, dtype=torch.float32, device="cuda")
    block_d[:, :n] = torch.from_numpy(_rows(7, R_ROWS, n)).cuda()
    D, A, ws, _, _ = _classify(O, ctx, oracle, win, frames[1], vs)
    assert 0 < D < n
    before_k, before_b = keys_d.clone(), block_d.clone()
    empty_k = torch.zeros(0, dtype=torch.int64, device="cuda")
    _, _, status = O.window_compact(ctx, keys_d, block_d, n, D - 1, empty_k, None, ws)
    torch.cuda.synchronize()
    assert int(status.item()) == 1
    assert torch.equal(keys_d, before_k) and torch.equal(block_d, before_b)
    with pytest.raises(A_.GslError):
        O.window_compact(ctx, keys_d, block_d, n, n + 1, empty_k, None, ws)
    too_many = torch.zeros(cap - n + D + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(A_.GslError):
        O.window_compact(ctx, keys_d, block_d, n, D, too_many,
                         torch.zeros(R_ROWS, too_many.shape[0], device="cuda"), ws)
    torch.cuda.synchronize()
    assert torch.equal(keys_d, before_k) and torch.equal(block_d, before_b)


def test_sliding_window_update_and_adam_on_capacity_layout(oracle):
    """SlidingWindow.update over three frames agrees with the oracle, and an
    Adam step on the capacity-strided block equals one on a contiguous copy."""
    O = ops()
    ctx = context()
    vs = 0.5
    n, P, cap = 6000, 5000, 12_000
    frames, means = S.lidar_stream(61, 4, P, n, extent=40.0, n_planes=150, range_m=12.0, step=1.0)
    sw = O.SlidingWindow(ctx, cap, vs)
    sw.keys[:n] = O.voxel_keys(ctx, torch.from_numpy(means).cuda(), vs)
    rows = _rows(8, R_ROWS, n)
    rows[14:] = 0.0
    sw.block[:, :n] = torch.from_numpy(rows).cuda()
    sw.n = n
    win_keys, win_rows = _okeys(oracle, means, vs), rows
    for f in range(1, 4):
        rng = np.random.default_rng(200 + f)
        made = {}

        def fetch(add_vox):
            made["vox"] = add_vox.numpy().view(np.uint64).copy()
            ak = np.repeat(made["vox"], 3)
            ar = rng.normal(size=(R_ROWS, len(ak))).astype(np.float32)
            ar[14:] = 0.0
            made["k"], made["r"] = ak, ar
            return torch.from_numpy(ak.view(np.int64).copy()), torch.from_numpy(ar)

        ek, er = sw.update(torch.from_numpy(frames[f]).cuda(), fetch)
        torch.cuda.synchronize()
        # the oracle's own classification decides its side; the GPU's ADD list must equal it
        pk, pok = oracle.voxel_key(frames[f], vs)
        _, add_o = oracle.window_classify(win_keys, pk, pok)
        assert np.array_equal(made["vox"], add_o)
        win_keys, win_rows, ek_w, er_w = oracle.window_maintain(win_keys, win_rows, pk[pok], np.repeat(add_o, 3),
                                                                made["r"])
        assert sw.n == len(win_keys)
        assert np.array_equal(_u64(sw.keys[:sw.n]), win_keys)
        assert np.array_equal(sw.block[:, :sw.n].cpu().numpy().view(np.uint32), win_rows.view(np.uint32))
        assert np.array_equal(_u64(ek), ek_w)
        assert np.array_equal(er.cpu().numpy().view(np.uint32), er_w.view(np.uint32))

    # Adam on the capacity layout (ld = capacity) against a contiguous copy
    N = sw.n
    st = sw.adam_state()
    dense = O.AdamState(sw.block[0:14, :N].contiguous(), sw.block[14:28, :N].contiguous(),
                        sw.block[28:42, :N].contiguous(), sw.d_step.clone())
    z = lambda *s: torch.zeros(*s, dtype=torch.float32, device="cuda")
    g1 = O.Gaussians(z(3, N), z(3, N), z(4, N), z(N), z(3, N))
    g2 = O.Gaussians(z(3, N), z(3, N), z(4, N), z(N), z(3, N))
    grads = O.Grads(N, 1, "cuda")
    gen = torch.Generator(device="cuda").manual_seed(9)
    for t in (grads.mean, grads.scale, grads.quat, grads.opacity, grads.color):
        t.copy_(torch.randn(t.shape, generator=gen, device="cuda"))
    hp = O.adam_hparams()
    O.adam_step(ctx, st, hp, grads, g1)
    O.adam_step(ctx, dense, hp, grads, g2)
    torch.cuda.synchronize()
    assert torch.equal(sw.block[0:14, :N], dense.raw) and torch.equal(sw.block[28:42, :N], dense.v)
    for k in ("mean", "scale", "quat", "opacity", "color"):
        assert torch.equal(getattr(g1, k), getattr(g2, k)), k


def test_window_transfer_pinned_staging():
    """gsl_window_transfer: keys and strided rows between device memory and
    pinned host memory, both directions, bit for bit; pageable host memory
    and wrong-side pointers are rejected on the host (nothing is copied)."""
    O = ops()
    A = O.A
    ctx = context()
    R, n = 42, 1000
    rng = np.random.default_rng(3)
    keys_h = torch.from_numpy(rng.integers(0, 2 ** 62, 3000, dtype=np.int64)).pin_memory()
    rows_h = torch.from_numpy(rng.normal(size=(R, 3000)).astype(np.float32)).pin_memory()
    keys_d = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    rows_d = torch.zeros(R, 1500, dtype=torch.float32, device="cuda")
    O.window_transfer(ctx, A.GSL_H2D, keys_h, rows_h, keys_d, rows_d, n)  # ld 3000 -> 1500
    torch.cuda.synchronize()
    assert torch.equal(keys_d.cpu(), keys_h[:n])
    assert torch.equal(rows_d[:, :n].cpu(), rows_h[:, :n])
    assert torch.all(rows_d[:, n:] == 0)
    back_k = torch.zeros(2000, dtype=torch.int64).pin_memory()
    back_r = torch.zeros(R, 2000, dtype=torch.float32).pin_memory()
    O.window_transfer(ctx, A.GSL_D2H, keys_d, rows_d, back_k, back_r, n)
    torch.cuda.synchronize()
    assert torch.equal(back_k[:n], keys_h[:n]) and torch.equal(back_r[:, :n], rows_h[:, :n])
    assert torch.all(back_r[:, n:] == 0) and torch.all(back_k[n:] == 0)
    # keys only, rows only, nothing
    O.window_transfer(ctx, A.GSL_D2H, keys_d, None, back_k, None, 10)
    O.window_transfer(ctx, A.GSL_H2D, None, rows_h, None, rows_d, 10)
    O.window_transfer(ctx, A.GSL_H2D, keys_h, rows_h, keys_d, rows_d, 0)
    torch.cuda.synchronize()
    # rejected before any copy: pageable host memory, device memory on the host side
    pageable = torch.zeros(n, dtype=torch.int64)
    for args in ((A.GSL_D2H, keys_d, None, pageable, None), (A.GSL_H2D, pageable, None, keys_d, None),
                 (A.GSL_D2H, keys_d, None, keys_d, None), (A.GSL_H2D, keys_h, None, keys_h, None)):
        with pytest.raises(A.GslError) as e:
            O.window_transfer(ctx, args[0], args[1], args[2], args[3], args[4], 10)
        assert e.value.code == A.GSL_EINVAL


def test_window_stream_through_host_map(oracle):
    """Six frames of a LiDAR stream that turns back: every evicted Gaussian
    goes to a host-side map (copied from the device through pinned memory),
    an ADD voxel the map holds gets its Gaussians back, others get new ones.
    The window (keys, 42 rows), the evicted Gaussians and the map agree bit
    for bit with the oracle's same sequence, and returning Gaussians come
    back with the rows they left with."""
    O = ops()
    ctx = context()
    vs = 0.5
    n, P, cap = 8000, 6000, 20_000
    frames, means = S.lidar_stream(41, 7, P, n, extent=40.0, n_planes=150, range_m=12.0, step=1.0)
    order = [1, 2, 3, 2, 1, 0]  # forward, then back over the same ground
    sw = O.SlidingWindow(ctx, cap, vs)
    win_keys = _okeys(oracle, means, vs)
    sw.keys[:n] = _dev(win_keys)
    win_rows = _rows(12, R_ROWS, n)
    sw.block[:, :n] = torch.from_numpy(win_rows).cuda()
    sw.n = n
    map_gpu, map_orc = {}, {}
    returned = 0
    for step, f in enumerate(order):
        rng = np.random.default_rng(400 + step)
        made = {}

        def fetch(add_vox):
            vox = add_vox.numpy().view(np.uint64)
            ks, rs = [], []
            for k in vox:
                if int(k) in map_gpu:
                    kk, rr = map_gpu.pop(int(k))
                else:
                    kk = np.repeat(k, 2)
                    rr = rng.normal(size=(R_ROWS, 2)).astype(np.float32)
                ks.append(kk)
                rs.append(rr)
            ak = np.concatenate(ks) if ks else np.zeros(0, np.uint64)
            ar = np.concatenate(rs, 1) if rs else np.zeros((R_ROWS, 0), np.float32)
            made["k"], made["r"] = ak, ar
            return torch.from_numpy(ak.view(np.int64).copy()), torch.from_numpy(ar)

        ek, er = sw.update(torch.from_numpy(frames[f]).cuda(), fetch)
        ek_np, er_np = _u64(ek).copy(), er.numpy().copy()
        for k in np.unique(ek_np):
            sel = ek_np == k
            assert int(k) not in map_gpu
            map_gpu[int(k)] = (ek_np[sel], er_np[:, sel])
        # the oracle: the same map logic on its own evictions
        pk, pok = oracle.voxel_key(frames[f], vs)
        _, add_o = oracle.window_classify(win_keys, pk, pok)
        ks, rs = [], []
        for k in add_o:
            if int(k) in map_orc:
                kk, rr = map_orc.pop(int(k))
                returned += len(kk)
            else:
                idx = np.nonzero(made["k"] == k)[0]  # new Gaussians: the rows the GPU side drew
                kk, rr = made["k"][idx], made["r"][:, idx]
            ks.append(kk)
            rs.append(rr)
        ak = np.concatenate(ks) if ks else np.zeros(0, np.uint64)
        ar = np.concatenate(rs, 1) if rs else np.zeros((R_ROWS, 0), np.float32)
        assert np.array_equal(ak, made["k"]) and np.array_equal(ar.view(np.uint32), made["r"].view(np.uint32))
        win_keys, win_rows, ek_w, er_w = oracle.window_maintain(win_keys, win_rows, pk[pok], ak, ar)
        for k in np.unique(ek_w):
            sel = ek_w == k
            map_orc[int(k)] = (ek_w[sel], er_w[:, sel])
        assert sw.n == len(win_keys)
        assert np.array_equal(_u64(sw.keys[:sw.n]), win_keys)
        assert np.array_equal(sw.block[:, :sw.n].cpu().numpy().view(np.uint32), win_rows.view(np.uint32))
        assert np.array_equal(ek_np, ek_w) and np.array_equal(er_np.view(np.uint32), er_w.view(np.uint32))
        assert sorted(map_gpu) == sorted(map_orc)
    assert returned > 0  # the stream turned back: some Gaussians came back from the map
