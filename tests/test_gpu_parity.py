"""GPU (HIP) path against the FP64 oracle, through the C ABI.

Bars (stated for the hot path): row index sets identical on >= 99.99% of
protons, and every voxel present on one side only lies where the oracle's
path passes within 1e-4 mm of that voxel's faces; path lengths within 1e-4
mm (1e-4 of the 1 mm voxel) on identical rows, any larger difference only
where the path runs within 1e-4 mm of a face of that voxel (a grazing
crossing); ||a_i||^2 within 1e-4 relative; images within 1e-3 relative L2
after a fixed number of sweeps.
"""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
from helpers import (check_mismatch_geometry, compare_rows, merge_rows, mismatch_voxels, oracle_geom,  # noqa: E402
                     oracle_grid, pct_args)
from paper_1707_05014_amd import _lib, api  # noqa: E402

LEN_TOL = 1e-4      # mm, on 1 mm voxels
IMG_TOL = 1e-3      # relative L2


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cfg1():
    cfg = synth.config(1)
    h = synth.generate(cfg)
    R = oracle.trace(oracle_grid(cfg), oracle_geom(cfg), h)
    return cfg, h, R


def _gpu_rows(cfg, h, len_dtype=0):
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    rows = api.mlp_trace(grid, geom, H, len_dtype=len_dtype)
    torch.cuda.synchronize()
    return grid, geom, H, rows


def _host_rows(rows, unit=1.0):
    rp = rows.row_ptr.cpu().numpy()
    idx = rows.idx[: rows.nnz].cpu().numpy()
    ln = rows.len[: rows.nnz].float().cpu().numpy().astype(np.float64) * unit
    n2 = rows.norm2.cpu().numpy()
    return rp, idx, ln, n2


def test_trace_parity_config1(cfg1):
    cfg, h, R = cfg1
    _say(f"trace parity: config 1, n={cfg.n}")
    grid, geom, H, rows = _gpu_rows(cfg, h)
    rp, idx, ln, n2 = _host_rows(rows)
    mp, mi, ml, dups = merge_rows(rp, idx, ln)
    assert dups == 0, "GPU rows must hold each voxel once"
    cmp = compare_rows(R.row_ptr, R.idx, R.len, mp, mi, ml)
    _say(f"  identical rows {cmp['frac_identical']:.6f}, max dlen {cmp['max_dlen']:.2e}, "
         f"max one-sided len {cmp['max_only_len']:.2e}, bad rows {cmp['bad_rows'][:10]}")
    assert cmp["frac_identical"] >= 0.9999
    assert cmp["frac_len_ok"] >= 0.9999
    cases = mismatch_voxels(R.row_ptr, R.idx, R.len, mp, mi, ml, LEN_TOL)
    bad, worst = check_mismatch_geometry(cfg, oracle_geom(cfg), h, np.arange(cfg.n), cases)
    _say(f"  {len(cases)} mismatched voxels; deepest one-sided penetration {worst:.2e} mm; outside the face "
         f"class: {bad[:5]}")
    assert len(cases) <= 400 and not bad
    ok = R.norm2 > 0
    assert np.array_equal(ok, n2 > 0)
    assert np.max(np.abs(n2[ok] - R.norm2[ok]) / R.norm2[ok]) <= 1e-4
    # path length per proton
    so = np.add.reduceat(R.len, R.row_ptr[:-1][ok]) if ok.any() else 0
    sg = np.add.reduceat(ml, mp[:-1][ok])
    assert np.max(np.abs(so - sg) / so) <= 1e-4


def test_trace_fp32_path_variant(cfg1):
    """Reduced-precision variant (FP32 path positions): its error against the
    oracle is reported; the bar is the per-proton path length (1e-4 relative)
    and that index differences stay slivers."""
    cfg, h, R = cfg1
    grid, geom = pct_args(cfg)
    geom.path_fp32 = 1
    H = api.Histories.from_numpy(h)
    rows = api.mlp_trace(grid, geom, H)
    rp, idx, ln, n2 = _host_rows(rows)
    mp, mi, ml, dups = merge_rows(rp, idx, ln)
    cmp = compare_rows(R.row_ptr, R.idx, R.len, mp, mi, ml)
    _say(f"FP32 path variant: identical rows {cmp['frac_identical']:.6f}, max dlen (identical rows) "
         f"{cmp['max_dlen']:.2e}, max dlen (all) {cmp['max_dlen_all']:.2e}, one-sided {cmp['max_only_len']:.2e}, "
         f"dups {dups}")
    ok = R.norm2 > 0
    so = np.add.reduceat(R.len, R.row_ptr[:-1][ok])
    sg = np.add.reduceat(ml, mp[:-1][ok])
    rel = np.abs(so - sg) / so
    _say(f"  rel path-length error: max {rel.max():.2e}, 99.9% {np.quantile(rel, 0.999):.2e}; "
         f"abs max {np.max(np.abs(so - sg)):.2e} mm")
    assert np.quantile(rel, 0.999) <= 1e-4
    assert np.max(np.abs(so - sg)) <= 1e-2
    assert cmp["frac_identical"] >= 0.99


def test_trace_f16_rows(cfg1):
    cfg, h, R = cfg1
    _say("trace f16 rows: config 1")
    grid, geom, H, rows32 = _gpu_rows(cfg, h, 0)
    rows16 = api.mlp_trace(grid, geom, H, len_dtype=1)
    torch.cuda.synchronize()
    assert rows16.nnz == rows32.nnz
    assert torch.equal(rows16.row_ptr, rows32.row_ptr)
    assert torch.equal(rows16.idx[: rows16.nnz], rows32.idx[: rows32.nnz])
    l32 = rows32.len[: rows32.nnz].double()
    l16 = rows16.len[: rows16.nnz].double()   # unit = 1 mm here
    # float16 rounding: half an ulp, 2^-11 relative for normal values and
    # 2^-25 absolute in the subnormal range below 2^-14
    bound = torch.clamp(l32 * 2.0 ** -11, min=2.0 ** -25) * (1 + 1e-6)
    assert torch.all(torch.abs(l16 - l32) <= bound)
    assert torch.equal(rows16.norm2, rows32.norm2)


def _run_oracle(cfg, h, R, algo, block, sweeps):
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    x, res = oracle.drop(R, h["wepl"], mask.astype(np.float64), order, block, cfg.lam, sweeps, mask=mask)
    return x, res, order, mask


def _run_gpu(cfg, h, algo, block, sweeps, order, mask, fused=False, len_dtype=0):
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    x = torch.from_numpy(mask.astype(np.float32)).cuda()
    params = api.sweep_params(algo, block, cfg.lam, sweeps, order=torch.from_numpy(order).cuda(),
                              hull_mask=torch.from_numpy(mask).cuda())
    rows = None if fused else api.mlp_trace(grid, geom, H, len_dtype=len_dtype)
    res = api.reconstruct(grid, geom, H, params, x, rows=rows)
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64), np.array(res)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_art_parity_config1(cfg1):
    """Config 1 as specified: hull start + 10 ART sweeps."""
    cfg, h, R = cfg1
    _say("ART parity: config 1, 10 sweeps")
    xo, ro, order, mask = _run_oracle(cfg, h, R, "art", 1, cfg.sweeps)
    xg, rg = _run_gpu(cfg, h, "art", 1, cfg.sweeps, order, mask)
    rel = _rel(xg, xo)
    _say(f"  image rel-L2 {rel:.2e}; residual oracle {ro[-1]:.4f} gpu {rg[-1]:.4f}")
    assert rel <= IMG_TOL
    assert np.allclose(rg, ro, rtol=1e-3)


@pytest.mark.parametrize("fused", [False, True], ids=["cached", "fused"])
def test_drop_parity_config1(cfg1, fused):
    cfg, h, R = cfg1
    _say(f"DROP parity: config 1, blocks of 5000, 6 sweeps, fused={fused}")
    xo, ro, order, mask = _run_oracle(cfg, h, R, "drop", 5000, 6)
    xg, rg = _run_gpu(cfg, h, "drop", 5000, 6, order, mask, fused=fused)
    rel = _rel(xg, xo)
    _say(f"  image rel-L2 {rel:.2e}; residuals oracle {ro[-1]:.4f} gpu {rg[-1]:.4f}")
    assert rel <= IMG_TOL
    assert np.allclose(rg, ro, rtol=1e-3)


def test_drop_ragged_blocks(cfg1):
    """Block size that leaves a short last block, several workgroups per block."""
    cfg, h, R = cfg1
    _say("DROP ragged blocks: 7777")
    xo, ro, order, mask = _run_oracle(cfg, h, R, "drop", 7777, 2)
    xg, rg = _run_gpu(cfg, h, "drop", 7777, 2, order, mask)
    assert _rel(xg, xo) <= IMG_TOL


def test_residual_at_known_image(cfg1):
    cfg, h, R = cfg1
    _say("residual at the truth image")
    truth = synth.truth_image(cfg)
    ro = oracle.residual(R, h["wepl"], truth.astype(np.float64))
    grid, geom, H, rows = _gpu_rows(cfg, h)
    xt = torch.from_numpy(truth).cuda()
    rc = api.residual(grid, geom, H, rows, xt)
    rf = api.residual(grid, geom, H, None, xt)
    assert rc == pytest.approx(ro, rel=1e-4)
    assert rf == pytest.approx(ro, rel=1e-4)


def test_roi_stats():
    _say("ROI stats")
    rng = np.random.default_rng(0)
    M = 100_003
    x = rng.normal(size=M).astype(np.float32)
    lab = rng.integers(0, 6, M).astype(np.uint8)
    s, c = api.roi_stats(torch.from_numpy(x).cuda(), torch.from_numpy(lab).cuda(), 5)
    means = (s.cpu().numpy() / c.cpu().numpy())
    assert np.allclose(means, oracle.roi_means(x, lab, 5), rtol=1e-9, atol=1e-12)
    assert np.array_equal(c.cpu().numpy(), np.bincount(lab, minlength=6)[1:])


def test_edge_cases():
    _say("edge cases: empty input, hull misses, NaN, row capacity")
    cfg = synth.config(1, n=2000)
    h = synth.generate(cfg)
    grid, geom = pct_args(cfg)
    # empty history set
    H0 = api.Histories({k: torch.empty(0, dtype=torch.float32, device="cuda") for k in api.FIELDS})
    r0 = api.mlp_trace(grid, geom, H0)
    assert r0.nnz == 0 and r0.row_ptr.cpu().tolist() == [0]
    # histories that miss the hull, and non-finite ones
    hb = {k: v.copy() for k, v in h.items()}
    hb["t_in"][:10] = 500.0
    hb["t_out"][:10] = 500.0
    hb["wepl"][10:13] = np.nan
    Hb = api.Histories.from_numpy(hb)
    with pytest.raises(_lib.PctError) as ei:
        api.mlp_trace(grid, geom, Hb)
    assert ei.value.code == _lib.PCT_ENONFINITE
    rows = api.mlp_trace(grid, geom, Hb, allow_nonfinite=True)
    cnt = np.diff(rows.row_ptr.cpu().numpy())
    assert np.all(cnt[:13] == 0) and np.mean(cnt[13:] > 0) > 0.99
    # capacity overflow: nothing but row_ptr written
    H = api.Histories.from_numpy(h)
    full = api.mlp_trace(grid, geom, H)
    small = api.Rows(torch.empty(cfg.n + 1, dtype=torch.int64, device="cuda"),
                     torch.full((10,), -7, dtype=torch.int32, device="cuda"),
                     torch.zeros(10, dtype=torch.float32, device="cuda"),
                     torch.zeros(cfg.n, dtype=torch.float64, device="cuda"), 0)
    with pytest.raises(_lib.PctError) as ei:
        api.mlp_trace(grid, geom, H, rows=small)
    assert ei.value.code == _lib.PCT_EROWCAP
    assert torch.all(small.idx == -7)
    assert torch.equal(small.row_ptr, full.row_ptr)


def test_fused_edge_cases():
    """Fused (rows rebuilt every sweep) with no histories, with an order
    entry out of range, and with non-finite histories (no path; the image
    stays finite)."""
    _say("fused edge cases")
    cfg = synth.config(1, n=3000)
    h = synth.generate(cfg)
    grid, geom = pct_args(cfg)
    mask = synth.hull_mask(cfg)
    tmask = torch.from_numpy(mask).cuda()
    # no histories: the sweeps leave the hull start, the residuals are 0
    H0 = api.Histories({k: torch.empty(0, dtype=torch.float32, device="cuda") for k in api.FIELDS})
    x = torch.from_numpy(mask.astype(np.float32)).cuda()
    res = api.reconstruct(grid, geom, H0, api.sweep_params("drop", 100, 0.5, 2, hull_mask=tmask), x)
    assert res == [0.0, 0.0]
    assert torch.equal(x, torch.from_numpy(mask.astype(np.float32)).cuda())
    # an order entry out of range is reported (the sweep reads the records through the order)
    H = api.Histories.from_numpy(h)
    bad = torch.arange(cfg.n, dtype=torch.int64, device="cuda")
    bad[17] = cfg.n + 5
    pb = api.sweep_params("drop", 1000, 0.5, 2, order=bad, hull_mask=tmask)
    with pytest.raises(_lib.PctError) as ei:
        api.reconstruct(grid, geom, H, pb, torch.from_numpy(mask.astype(np.float32)).cuda())
    assert ei.value.code == _lib.PCT_EINVAL
    # non-finite histories get no path: same image as without them
    hn = {k: v.copy() for k, v in h.items()}
    hn["wepl"][5:9] = np.nan
    hn["phi"][20] = np.inf
    keep = np.ones(cfg.n, bool)
    keep[[5, 6, 7, 8, 20]] = False
    xa = torch.from_numpy(mask.astype(np.float32)).cuda()
    api.reconstruct(grid, geom, api.Histories.from_numpy(hn), api.sweep_params("drop", cfg.n, 0.5, 1, hull_mask=tmask),
                    xa)
    xb = torch.from_numpy(mask.astype(np.float32)).cuda()
    api.reconstruct(grid, geom, api.Histories.from_numpy({k: v[keep].copy() for k, v in h.items()}),
                    api.sweep_params("drop", cfg.n, 0.5, 1, hull_mask=tmask), xb)
    torch.cuda.synchronize()
    assert torch.isfinite(xa).all()
    assert _rel(xa.cpu().numpy().astype(np.float64), xb.cpu().numpy().astype(np.float64)) <= 1e-6


def test_fused_equals_cached_single_block(cfg1):
    """The fused sweep and the cached sweep see the same rows: one DROP block
    over every proton gives the same update up to atomic summation order."""
    cfg, h, R = cfg1
    _say("fused vs cached, one block")
    order = np.arange(cfg.n, dtype=np.int64)
    mask = synth.hull_mask(cfg)
    xa, _ = _run_gpu(cfg, h, "drop", cfg.n, 1, order, mask, fused=False)
    xb, _ = _run_gpu(cfg, h, "drop", cfg.n, 1, order, mask, fused=True)
    assert _rel(xa, xb) <= 1e-6


def test_fused_kept_counts_match_counting(cfg1):
    """A fused reconstruction of several sweeps keeps each block's voxel
    counts from its first sweep; one-sweep calls count with atomics every
    time.  Both give the same image up to atomic summation order, and the
    kept counts need the larger workspace (a smaller one falls back)."""
    cfg, h, R = cfg1
    _say("fused: kept block counts vs counting every sweep")
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    xa, ra = _run_gpu(cfg, h, "drop", 7000, 4, order, mask, fused=True)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    x = torch.from_numpy(mask.astype(np.float32)).cuda()
    p1 = api.sweep_params("drop", 7000, cfg.lam, 1, order=torch.from_numpy(order).cuda(),
                          hull_mask=torch.from_numpy(mask).cuda())
    for _ in range(4):
        api.project_sweep(grid, geom, H, None, x, p1)
    xb = x.cpu().numpy().astype(np.float64)
    assert _rel(xa, xb) <= 1e-6
    lib = _lib.load()
    p4 = api.sweep_params("drop", 7000, cfg.lam, 4)
    big = lib.pct_workspace_size(ctypes.byref(grid), None, ctypes.byref(p4.struct), cfg.n, 1)
    small = lib.pct_workspace_size(ctypes.byref(grid), None, None, cfg.n, 1)
    n_blocks = -(-cfg.n // 7000)
    assert big - small >= n_blocks * cfg.grid.M * 2


@pytest.mark.parametrize("block,scale", [(100_000, 1.0), (7000, 16.0)], ids=["one-block", "b-x16"])
def test_fused_packed_counting_sweep(cfg1, block, scale):
    """A fused sweep that forms the block counts adds each entry's numerator
    and count with one packed 64-bit atomic (fixed point, 2^-27 for a block
    of 1e5 rows) when the workspace holds every history's path record;
    contributions of 4 or more take separate FP32 and count atomics instead (b
    x 16 makes many of them).  Against the same sweeps with a workspace too
    small for the records (then every entry takes the separate atomics), up
    to rounding, and against the oracle."""
    cfg, h, R = cfg1
    h2 = dict(h)
    h2["wepl"] = (h["wepl"] * scale).astype(h["wepl"].dtype)
    _say(f"fused: packed counting sweeps, blocks of {block}, b x {scale}")
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h2)
    p1 = api.sweep_params("drop", block, cfg.lam, 1, order=torch.from_numpy(order).cuda(),
                          hull_mask=torch.from_numpy(mask).cuda())
    xa = torch.from_numpy(mask.astype(np.float32)).cuda()
    for _ in range(2):
        api.project_sweep(grid, geom, H, None, xa, p1)  # workspace sized for the fused form: packed
    lib = _lib.load()
    small = lib.pct_workspace_size(ctypes.byref(grid), None, None, cfg.n, 0)
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    xb = torch.from_numpy(mask.astype(np.float32)).cuda()
    hs = H.struct()
    for _ in range(2):
        code = lib.pct_project_sweep(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), None, xb.data_ptr(),
                                     ctypes.byref(p1.struct), None, ws.data_ptr(), small,
                                     torch.cuda.current_stream().cuda_stream)
        assert code == _lib.PCT_OK
    torch.cuda.synchronize()
    ga, gb = xa.cpu().numpy().astype(np.float64), xb.cpu().numpy().astype(np.float64)
    rel = _rel(ga, gb)
    _say(f"  image rel-L2 packed vs separate atomics: {rel:.2e}")
    assert rel <= 1e-6
    xo, ro = oracle.drop(R, h2["wepl"], mask.astype(np.float64), order, block, cfg.lam, 2, mask=mask)
    assert _rel(ga, xo) <= IMG_TOL
    # the several-sweep reconstruction (block counts kept after the first sweep) agrees too
    xc, _ = _run_gpu(cfg, h2, "drop", block, 2, order, mask, fused=True)
    assert _rel(xc, gb) <= 1e-6


def test_fused_chunked_setup_matches(cfg1):
    """With a workspace too small for one path record per history the fused
    sweep sets up each block's protons just before projecting them; the
    image equals the one-record-per-history form up to atomic order."""
    cfg, h, R = cfg1
    _say("fused: records per block vs per history")
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    p1 = api.sweep_params("drop", 7000, cfg.lam, 1, order=torch.from_numpy(order).cuda(),
                          hull_mask=torch.from_numpy(mask).cuda())
    xa = torch.from_numpy(mask.astype(np.float32)).cuda()
    api.project_sweep(grid, geom, H, None, xa, p1)  # workspace sized for the fused form
    lib = _lib.load()
    small = lib.pct_workspace_size(ctypes.byref(grid), None, None, cfg.n, 0)
    full = lib.pct_workspace_size(ctypes.byref(grid), None, None, cfg.n, 1)
    assert full - small >= (cfg.n - min(cfg.n, 1 << 20)) * 128
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    xb = torch.from_numpy(mask.astype(np.float32)).cuda()
    hs = H.struct()
    res = torch.empty(1, dtype=torch.float64, device="cuda")
    code = lib.pct_project_sweep(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), None, xb.data_ptr(),
                                 ctypes.byref(p1.struct), res.data_ptr(), ws.data_ptr(), small,
                                 torch.cuda.current_stream().cuda_stream)
    assert code == _lib.PCT_OK
    torch.cuda.synchronize()
    ra = api.residual(grid, geom, H, None, xa)
    assert _rel(xa.cpu().numpy().astype(np.float64), xb.cpu().numpy().astype(np.float64)) <= 1e-6
    assert abs(float(res.item()) - ra) <= 1e-6 * ra


def test_fused_workspace_forms_agree():
    """pct_reconstruct (fused, 2 sweeps) with three workspace sizes: one path
    record per history and the kept block counts; the counts but per-block
    set-up (the records do not fit); neither.  Same image up to atomic
    order.  Needs more than 2^20 histories so that the forms differ."""
    n = (1 << 20) + 150_000
    _say(f"fused workspace forms: {n} histories on the small grid")
    cfg = synth.config(1, n=n)
    h = synth.generate(cfg)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    mask = synth.hull_mask(cfg)
    order = torch.from_numpy(synth.block_order(n, cfg.perm_seed)).cuda()
    p = api.sweep_params("drop", 200_000, 0.5, 2, order=order, hull_mask=torch.from_numpy(mask).cuda())
    lib = _lib.load()
    full = lib.pct_workspace_size(ctypes.byref(grid), None, ctypes.byref(p.struct), n, 1)
    counts_only = full - (n - (1 << 20)) * 128
    minimal = lib.pct_workspace_size(ctypes.byref(grid), None, None, n, 0)
    assert minimal < counts_only < full
    images, resids = [], []
    for size in (full, counts_only, minimal):
        ws = torch.empty(size, dtype=torch.uint8, device="cuda")
        x = torch.from_numpy(mask.astype(np.float32)).cuda()
        res = (ctypes.c_double * 2)()
        hs = H.struct()
        code = lib.pct_reconstruct(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), ctypes.byref(p.struct),
                                   None, None, x.data_ptr(), res, ws.data_ptr(), size,
                                   torch.cuda.current_stream().cuda_stream)
        assert code == _lib.PCT_OK, lib.pct_last_error()
        torch.cuda.synchronize()
        images.append(x.cpu().numpy().astype(np.float64))
        resids.append([res[0], res[1]])
        del ws
    for im, rs in zip(images[1:], resids[1:]):
        assert _rel(im, images[0]) <= 1e-6
        assert np.allclose(rs, resids[0], rtol=1e-6)


# ------------------------------------------------------------- tiled plan
def _plan_run(cfg, h, block, sweeps, order, mask, len_dtype=0, via_reconstruct=True):
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    x = torch.from_numpy(mask.astype(np.float32)).cuda()
    params = api.sweep_params("drop", block, cfg.lam, sweeps, order=torch.from_numpy(order).cuda(),
                              hull_mask=torch.from_numpy(mask).cuda())
    rows = api.mlp_trace(grid, geom, H, len_dtype=len_dtype)
    plan = api.plan_build(grid, H, rows, params)
    if via_reconstruct:
        res = api.reconstruct(grid, geom, H, params, x, rows=rows, plan=plan)
    else:
        p1 = api.sweep_params("drop", block, cfg.lam, 1, order=params.order, hull_mask=params.hull_mask)
        res = []
        for _ in range(sweeps):
            api.plan_sweep(grid, plan, x, p1)
            res.append(api.plan_residual(grid, plan, x))
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64), np.array(res), plan, rows


@pytest.mark.parametrize("via", [True, False], ids=["reconstruct", "sweeps"])
def test_plan_drop_parity_config1(cfg1, via):
    cfg, h, R = cfg1
    _say(f"plan DROP parity: config 1, blocks of 5000, 6 sweeps, via_reconstruct={via}")
    xo, ro, order, mask = _run_oracle(cfg, h, R, "drop", 5000, 6)
    xg, rg, plan, _ = _plan_run(cfg, h, 5000, 6, order, mask, via_reconstruct=via)
    s = plan.struct
    _say(f"  plan: entries {s.entries} chunks {s.chunks} refs {s.refs} max_chunks {s.max_chunks} "
         f"max_ends {s.max_ends} bytes {s.bytes}")
    rel = _rel(xg, xo)
    _say(f"  image rel-L2 {rel:.2e}; residual oracle {ro[-1]:.4f} gpu {rg[-1]:.4f}")
    assert rel <= IMG_TOL
    assert np.allclose(rg, ro, rtol=1e-3)


def test_plan_ragged_grid_and_blocks():
    """Grid dimensions that are not multiples of the 16 x 16 x 8 tile, and a
    block size that leaves a short last block."""
    cfg = synth.config(1, n=60000)
    cfg.grid = synth.Grid(60, 62, 14, 1.0, 1.0, 1.0, -30.0, -31.0, -7.0)
    h = synth.generate(cfg)
    _say("plan ragged: grid 60x62x14, blocks of 7777")
    R = oracle.trace(oracle_grid(cfg), oracle_geom(cfg), h)
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    xo, ro = oracle.drop(R, h["wepl"], mask.astype(np.float64), order, 7777, cfg.lam, 3, mask=mask)
    xg, rg, plan, _ = _plan_run(cfg, h, 7777, 3, order, mask)
    assert _rel(xg, xo) <= IMG_TOL
    assert np.allclose(rg, ro, rtol=1e-3)


def test_plan_long_lists(cfg1):
    """One block of all 1e5 rows: the longest tile lists (each list is summed
    by one workgroup) and the smallest fixed-point scale of the update (2^41
    for a block of 1e5 rows), checked against the oracle."""
    cfg, h, R = cfg1
    _say("plan with one block of 100000 rows")
    xo, ro, order, mask = _run_oracle(cfg, h, R, "drop", cfg.n, 3)
    xg, rg, plan, _ = _plan_run(cfg, h, cfg.n, 3, order, mask)
    s = plan.struct
    _say(f"  plan: entries {s.entries} piece ends {s.ends} tiles {s.n_tiles}")
    assert s.entries / s.n_tiles > 1e5  # long lists, on average
    rel = _rel(xg, xo)
    _say(f"  image rel-L2 {rel:.2e}")
    assert rel <= IMG_TOL
    assert np.allclose(rg, ro, rtol=1e-3)


def test_plan_large_contributions(cfg1):
    """b scaled by 16, so that many contributions r_i a_ij reach the
    magnitude (16) above which the update adds them in float32 instead of
    fixed point: both kinds of sum in one image, against the oracle run on the
    same scaled b."""
    cfg, h, R = cfg1
    h2 = dict(h)
    h2["wepl"] = (h["wepl"] * 16.0).astype(h["wepl"].dtype)
    _say("plan with b x 16 (contributions beyond the fixed-point range)")
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    xo, ro = oracle.drop(R, h2["wepl"], mask.astype(np.float64), order, 5000, cfg.lam, 2, mask=mask)
    xg, rg, plan, rows = _plan_run(cfg, h2, 5000, 2, order, mask)
    # share of entries whose first-sweep contribution is 16 or more (from the oracle's rows)
    rp, idx, ln = R.row_ptr, R.idx, R.len
    x0 = mask.astype(np.float64)
    q = order[:5000]
    big = 0
    tot = 0
    for i in q:
        a, b = rp[i], rp[i + 1]
        if b == a:
            continue
        n2 = float(np.dot(ln[a:b], ln[a:b]))
        r = (h2["wepl"][i] - float(np.dot(ln[a:b], x0[idx[a:b]]))) / n2
        big += int(np.count_nonzero(np.abs(r * ln[a:b]) >= 16.0))
        tot += b - a
    rel = _rel(xg, xo)
    _say(f"  first block: {big} of {tot} contributions >= 16; image rel-L2 {rel:.2e}")
    assert 0.01 * tot < big < 0.99 * tot
    assert rel <= IMG_TOL
    assert np.allclose(rg, ro, rtol=1e-3)


def test_plan_sweep_reproducible(cfg1):
    """The update's sums are exact integers, so two sweeps from the same image
    give the same bits, whatever order the entries' additions took."""
    cfg, h, R = cfg1
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    order = torch.from_numpy(synth.block_order(cfg.n, cfg.perm_seed)).cuda()
    mask = torch.from_numpy(synth.hull_mask(cfg)).cuda()
    params = api.sweep_params("drop", 5000, cfg.lam, 1, order=order, hull_mask=mask)
    rows = api.mlp_trace(grid, geom, H)
    plan = api.plan_build(grid, H, rows, params)
    outs = []
    for _ in range(3):
        x = mask.to(torch.float32)
        api.plan_sweep(grid, plan, x, params)
        api.plan_sweep(grid, plan, x, params)
        outs.append(x.cpu().numpy())
    torch.cuda.synchronize()
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    assert np.array_equal(outs[0].view(np.uint32), outs[2].view(np.uint32))


def test_plan_f16_rows_match_csr(cfg1):
    """FP16-length plan against the FP16-length CSR path (same matrix)."""
    cfg, h, R = cfg1
    _say("plan with FP16 rows vs CSR path with FP16 rows")
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    xa, _ = _run_gpu(cfg, h, "drop", 5000, 3, order, mask, len_dtype=1)
    xb, _, _, _ = _plan_run(cfg, h, 5000, 3, order, mask, len_dtype=1)
    assert _rel(xb, xa) <= 1e-5
    # and the FP16 form against the FP64 oracle: stated, bounded loosely
    xo, _, _, _ = _run_oracle(cfg, h, R, "drop", 5000, 3)
    _say(f"  FP16 rows vs oracle: rel-L2 {_rel(xb, xo):.2e}")
    assert _rel(xb, xo) <= 1e-2


def test_plan_rejects_mismatched_params(cfg1):
    cfg, h, R = cfg1
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    order = torch.from_numpy(synth.block_order(cfg.n, cfg.perm_seed)).cuda()
    params = api.sweep_params("drop", 5000, 0.5, 1, order=order)
    rows = api.mlp_trace(grid, geom, H)
    plan = api.plan_build(grid, H, rows, params)
    x = torch.zeros(cfg.grid.M, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.PctError) as ei:
        api.plan_sweep(grid, plan, x, api.sweep_params("drop", 4000, 0.5, 1, order=order))
    assert ei.value.code == _lib.PCT_EINVAL
    with pytest.raises(_lib.PctError):
        api.plan_build(grid, H, rows, api.sweep_params("drop", 300_000, 0.5, 1, order=order))
