"""Shared test helpers: turn a synthetic workload into oracle arguments."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def oracle_grid(cfg: synth.Config) -> oracle.OrcGrid:
    g = cfg.grid
    return oracle.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)


def oracle_geom(cfg: synth.Config, poly=None, highland_log: bool = True, step: float | None = None):
    b = cfg.phantom.body
    poly = synth.prior_poly(cfg.beam.E_kin) if poly is None else poly
    return oracle.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1,
                            min(cfg.grid.dx, cfg.grid.dy, cfg.grid.dz) if step is None else step,
                            poly, highland_log=highland_log)


def hist_row(h: dict, i: int) -> np.ndarray:
    return np.array([h[k][i] for k in oracle.FIELDS], dtype=np.float64)


# ----------------------------------------------------------------- GPU side
def pct_args(cfg: synth.Config, poly=None, highland_log: bool = True, step: float | None = None):
    """(pct_grid, pct_geom) of a workload for the HIP library."""
    from paper_1707_05014_amd import api
    g = cfg.grid
    b = cfg.phantom.body
    poly = synth.prior_poly(cfg.beam.E_kin) if poly is None else poly
    grid = api.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
    geom = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1,
                         min(g.dx, g.dy, g.dz) if step is None else step, poly, highland_log=highland_log)
    return grid, geom


def merge_rows(row_ptr, idx, ln):
    """Per-row sort by voxel and sum of equal voxels (host, numpy).
    Returns (row_ptr, idx, len, dup_count)."""
    row_ptr = np.asarray(row_ptr, np.int64)
    n = len(row_ptr) - 1
    rid = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    key = rid * (1 << 31) + np.asarray(idx, np.int64)
    o = np.argsort(key, kind="stable")
    key = key[o]
    ln = np.asarray(ln, np.float64)[o]
    uk, first = np.unique(key, return_index=True)
    sums = np.add.reduceat(ln, first) if len(ln) else ln
    dups = len(key) - len(uk)
    r = uk >> 31
    new_ptr = np.zeros(n + 1, np.int64)
    np.add.at(new_ptr, r + 1, 1)
    return np.cumsum(new_ptr), (uk & ((1 << 31) - 1)).astype(np.int32), sums, dups


def compare_rows(o_ptr, o_idx, o_len, g_ptr, g_idx, g_len, len_tol=1e-4):
    """Compare two sets of fully merged, voxel-sorted rows.
    Returns dict: frac_identical (index sets), mismatch rows, max |dlen| on
    common voxels of identical rows, max length of a voxel present on one side
    only, and frac_len_ok: the share of the rows with identical index sets
    whose every length is within len_tol."""
    n = len(o_ptr) - 1
    ro = np.repeat(np.arange(n, dtype=np.int64), np.diff(o_ptr))
    rg = np.repeat(np.arange(n, dtype=np.int64), np.diff(g_ptr))
    ko = ro * (1 << 31) + o_idx.astype(np.int64)
    kg = rg * (1 << 31) + g_idx.astype(np.int64)
    in_g = np.isin(ko, kg, assume_unique=True)
    in_o = np.isin(kg, ko, assume_unique=True)
    bad_rows = np.union1d(ro[~in_g], rg[~in_o])
    good = np.ones(n, bool)
    good[bad_rows] = False
    # lengths on common voxels (both arrays sorted by key, so the common parts align)
    lo = o_len[in_g]
    lg = g_len[in_o]
    common_rows = ro[in_g]
    d = np.abs(lo - lg)
    max_d_good = float(d[good[common_rows]].max()) if np.any(good[common_rows]) else 0.0
    only = np.concatenate([o_len[~in_g], g_len[~in_o]])
    ok = good.copy()
    ok[np.unique(common_rows[d > len_tol])] = False
    n_good = int(good.sum())
    return dict(frac_identical=float(good.mean()) if n else 1.0, bad_rows=bad_rows,
                frac_len_ok=float(ok.sum()) / n_good if n_good else 1.0,
                max_dlen=max_d_good, max_dlen_all=float(d.max()) if len(d) else 0.0,
                max_only_len=float(only.max()) if len(only) else 0.0)


# ------------------------------------------------- geometry of row mismatches
FACE_TOL = 1e-4     # mm: how close to a voxel face a path must pass for a mismatch to be allowed
GRAZE_LEN = 0.1     # mm of path within FACE_TOL of one face: a crossing at a sine <= 2e-3


def polyline_xyz(geom, hist_row) -> np.ndarray:
    """The oracle's most-likely-path polyline of one history, object frame (n x 3)."""
    u, t, v = oracle.mlp_path(geom, hist_row)
    c, s = np.cos(hist_row[0]), np.sin(hist_row[0])
    return np.stack([u * c - t * s, u * s + t * c, v], axis=1)


def voxel_box(cfg: synth.Config, j: int):
    g = cfg.grid
    i, jj, k = j % g.nx, (j // g.nx) % g.ny, j // (g.nx * g.ny)
    lo = np.array([g.ox + i * g.dx, g.oy + jj * g.dy, g.oz + k * g.dz])
    return lo, lo + np.array([g.dx, g.dy, g.dz])


def signed_depth(p, lo, hi):
    """Distance from p to the box surface, positive inside, negative outside
    (a concave function along any line, since the box is convex)."""
    p = np.asarray(p, np.float64)
    ins = np.minimum(p - lo, hi - p).min(axis=-1)
    out = np.linalg.norm(np.maximum(np.maximum(lo - p, p - hi), 0.0), axis=-1)
    return np.where(ins >= 0.0, ins, -out)


def _segments_near(xyz, lo, hi, pad: float):
    """Segments of the polyline whose bounding boxes meet the box grown by pad."""
    P, Q = xyz[:-1], xyz[1:]
    bl, bh = np.minimum(P, Q), np.maximum(P, Q)
    hit = np.all((bh >= lo - pad) & (bl <= hi + pad), axis=1)
    return P[hit], Q[hit]


def max_penetration(xyz, lo, hi, iters: int = 90, pad: float = 1.0) -> float:
    """max over the polyline of signed_depth: how deep the path enters the box
    (negative: how far it stays outside; -inf beyond pad).  Ternary search per
    segment on the concave depth profile."""
    best = -np.inf
    for P, Q in zip(*_segments_near(np.asarray(xyz, np.float64), lo, hi, pad)):
        a, b = 0.0, 1.0
        for _ in range(iters):
            m1, m2 = a + (b - a) / 3.0, b - (b - a) / 3.0
            if signed_depth(P + m1 * (Q - P), lo, hi) < signed_depth(P + m2 * (Q - P), lo, hi):
                a = m1
            else:
                b = m2
        s = 0.5 * (a + b)
        best = max(best, float(signed_depth(P + s * (Q - P), lo, hi)), float(signed_depth(P, lo, hi)),
                   float(signed_depth(Q, lo, hi)))
    return best


def near_face_length(xyz, lo, hi, tol: float = FACE_TOL, h: float = 2e-5) -> float:
    """Largest length of path, over the six faces of the box, that lies within
    tol of the face's plane and within tol of the face itself (sampled every
    h mm).  A crossing of the face at an angle of sine sin_t gives about
    2 tol / sin_t; a path running along the face gives its whole length."""
    best = 0.0
    span = np.stack([lo, hi])
    for P, Q in zip(*_segments_near(np.asarray(xyz, np.float64), lo, hi, tol)):
        seg = float(np.linalg.norm(Q - P))
        if seg == 0.0:
            continue
        s = np.linspace(0.0, 1.0, max(2, int(np.ceil(seg / h)) + 1))
        pts = P[None, :] + s[:, None] * (Q - P)[None, :]
        for a in range(3):
            o = [q for q in range(3) if q != a]
            within = np.all((pts[:, o] >= lo[o] - tol) & (pts[:, o] <= hi[o] + tol), axis=1)
            for side in range(2):
                near = within & (np.abs(pts[:, a] - span[side, a]) <= tol)
                best = max(best, float(near.sum()) * seg / (len(s) - 1))
    return best


def mismatch_voxels(o_ptr, o_idx, o_len, g_ptr, g_idx, g_len, len_tol: float = 1e-4):
    """(row, voxel, kind, dlen) for every voxel present in one row set only
    (kind 'oracle' / 'gpu') or present in both with lengths more than len_tol
    apart (kind 'length'); rows fully merged and sorted by voxel."""
    n = len(o_ptr) - 1
    ro = np.repeat(np.arange(n, dtype=np.int64), np.diff(o_ptr))
    rg = np.repeat(np.arange(n, dtype=np.int64), np.diff(g_ptr))
    ko = ro * (1 << 31) + np.asarray(o_idx, np.int64)
    kg = rg * (1 << 31) + np.asarray(g_idx, np.int64)
    in_g = np.isin(ko, kg, assume_unique=True)
    in_o = np.isin(kg, ko, assume_unique=True)
    out = []
    for k, ln in zip(ko[~in_g], np.asarray(o_len)[~in_g]):
        out.append((int(k >> 31), int(k & ((1 << 31) - 1)), "oracle", float(ln)))
    for k, ln in zip(kg[~in_o], np.asarray(g_len)[~in_o]):
        out.append((int(k >> 31), int(k & ((1 << 31) - 1)), "gpu", float(ln)))
    d = np.asarray(g_len)[in_o] - np.asarray(o_len)[in_g]
    kc = ko[in_g]
    for k, dl in zip(kc[np.abs(d) > len_tol], d[np.abs(d) > len_tol]):
        out.append((int(k >> 31), int(k & ((1 << 31) - 1)), "length", float(dl)))
    return out


def check_mismatch_geometry(cfg, geom, h: dict, rows_sel, cases, limit: int = 400):
    """Every mismatch must sit where the oracle's path passes within FACE_TOL
    of a voxel face: a one-sided voxel is entered (or missed) by at most
    FACE_TOL; a length difference on a common voxel needs the path to run
    within FACE_TOL of one of its faces over at least GRAZE_LEN.  rows_sel
    maps the row numbers of `cases` to history indices.  Returns the list of
    violations (empty when all hold) and the worst penetration seen."""
    bad = []
    worst = 0.0
    for (r, j, kind, val) in cases[:limit]:
        i = int(rows_sel[r])
        xyz = polyline_xyz(geom, hist_row(h, i))
        lo, hi = voxel_box(cfg, j)
        if kind in ("oracle", "gpu"):
            pen = max_penetration(xyz, lo, hi)
            worst = max(worst, abs(pen))
            if abs(pen) > FACE_TOL:
                bad.append((i, j, kind, val, pen))
        else:
            nl = near_face_length(xyz, lo, hi)
            if nl < GRAZE_LEN:
                bad.append((i, j, kind, val, nl))
    return bad, worst
