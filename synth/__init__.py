"""Seeded synthetic inputs: phantoms, proton histories, block orders.

This module only produces input data.  It holds none of the reconstruction's
arithmetic (no most-likely path, no voxel traversal, no projection), so the
FP64 oracle and the GPU path can both consume what it makes without sharing
any of the method's code.

The workloads stand in for the paper's scanner data (Sec. 3 and Sec. 4: a
head-sized phantom with cylindrical inserts of known RSP, 200 MeV protons,
N of order 10^8-10^9 histories, M of order 10^6 voxels, Sec. 2), which is not
available here.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libpctgen.so")

HIST_FIELDS = ("phi", "t_in", "v_in", "dt_in", "dv_in", "t_out", "v_out", "dt_out", "dv_out", "wepl")


_SO_GPU = os.path.join(_HERE, "libpctgen_hip.so")


def build(force: bool = True) -> str:
    """Compile the host generator with gcc (FP64, OpenMP, no fast-math) and
    the device generator with hipcc for gfx950."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp",
               os.path.join(_HERE, "gen.c"), "-lm"]
        subprocess.check_call(cmd)
        os.replace(_SO + ".tmp", _SO)
    if force or not os.path.exists(_SO_GPU):
        hipcc = os.environ.get("HIPCC") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc")
        arch = os.environ.get("PCT_OFFLOAD_ARCH", "gfx950")
        cmd = [hipcc, "-O3", "-std=c++17", f"--offload-arch={arch}", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-o", _SO_GPU + ".tmp", os.path.join(_HERE, "gen_gpu.hip")]
        subprocess.check_call(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        os.replace(_SO_GPU + ".tmp", _SO_GPU)
    return _SO


class _Shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("c", ctypes.c_double * 3), ("ax", ctypes.c_double * 3),
                ("yaw", ctypes.c_double), ("z0", ctypes.c_double), ("z1", ctypes.c_double),
                ("delta_rsp", ctypes.c_double), ("bound_r", ctypes.c_double), ("cy", ctypes.c_double),
                ("sy", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("n_angles", ctypes.c_int32), ("t_half", ctypes.c_double), ("v_half", ctypes.c_double),
                ("slope_sigma", ctypes.c_double), ("u_in", ctypes.c_double), ("u_out", ctypes.c_double),
                ("step", ctypes.c_double), ("E_kin", ctypes.c_double), ("bk_alpha", ctypes.c_double),
                ("bk_p", ctypes.c_double), ("m_p", ctypes.c_double), ("E0_hl", ctypes.c_double),
                ("X0", ctypes.c_double), ("highland_log", ctypes.c_int32), ("scatter", ctypes.c_int32),
                ("wepl_sigma", ctypes.c_double), ("body_rxy", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        fp = ctypes.POINTER(ctypes.c_float)
        lib.pctgen_histories.restype = ctypes.c_int64
        lib.pctgen_histories.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(_Shape), ctypes.c_int32,
                                         ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64] + [fp] * 10 + [
                                            ctypes.c_int32]
        lib.pctgen_miss_histories.restype = ctypes.c_int64
        lib.pctgen_miss_histories.argtypes = lib.pctgen_histories.argtypes
        lib.pctgen_segment_wepl.restype = ctypes.c_double
        lib.pctgen_segment_wepl.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        lib.pctgen_point_rsp.restype = ctypes.c_double
        lib.pctgen_point_rsp.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        lib.pctgen_truth_image.restype = None
        lib.pctgen_truth_image.argtypes = [ctypes.POINTER(_Shape), ctypes.c_int32] + [ctypes.c_int32] * 3 + [
            ctypes.c_double] * 6 + [ctypes.c_int32, fp, ctypes.c_int32]
        lib.pctgen_permutation.restype = None
        lib.pctgen_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64)]
        lib.pctgen_philox4x32_10.restype = None
        lib.pctgen_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32),
                                             ctypes.POINTER(ctypes.c_uint32)]
        _lib = lib
    return _lib


def default_threads() -> int:
    """Every core this process may run on, limited by OMP_NUM_THREADS."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


# ----------------------------------------------------------------- geometry
@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    ox: float = 0.0
    oy: float = 0.0
    oz: float = 0.0

    @property
    def M(self) -> int:
        return self.nx * self.ny * self.nz

    def centers(self):
        i = np.arange(self.nx)
        j = np.arange(self.ny)
        k = np.arange(self.nz)
        cx = self.ox + (i + 0.5) * self.dx
        cy = self.oy + (j + 0.5) * self.dy
        cz = self.oz + (k + 0.5) * self.dz
        Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
        return X.ravel(), Y.ravel(), Z.ravel()


@dataclass
class Shape:
    kind: int            # 0 ellipsoid, 1 elliptic z-cylinder
    c: tuple
    ax: tuple
    yaw: float
    z0: float
    z1: float
    rsp: float           # absolute RSP of the material


@dataclass
class Phantom:
    body: Shape                         # elliptic cylinder: also the reconstruction hull
    inserts: list = field(default_factory=list)

    def shapes_c(self):
        arr = (_Shape * (1 + len(self.inserts)))()
        allsh = [self.body] + list(self.inserts)
        for n, s in enumerate(allsh):
            arr[n].kind = s.kind
            for q in range(3):
                arr[n].c[q] = s.c[q]
                arr[n].ax[q] = s.ax[q]
            arr[n].yaw = s.yaw
            arr[n].z0 = s.z0
            arr[n].z1 = s.z1
            arr[n].delta_rsp = s.rsp if n == 0 else s.rsp - self.body.rsp
            if s.kind == 0:
                br = max(s.ax)
            else:
                br = math.hypot(max(s.ax[0], s.ax[1]), max(abs(s.z0 - s.c[2]), abs(s.z1 - s.c[2])))
            arr[n].bound_r = br + 1e-6
        return arr, len(allsh)


@dataclass
class Beam:
    n_angles: int
    t_half: float
    v_half: float
    slope_sigma: float
    u_in: float
    u_out: float
    E_kin: float = 200.0
    step: float = 1.0
    wepl_sigma: float = 0.5
    scatter: bool = True
    highland_log: bool = True


# physical constants of the synthetic physics and the path prior
M_PROTON = 938.272          # MeV
E0_HIGHLAND = 13.6          # MeV
X0_WATER = 360.8            # mm
BK_ALPHA = 0.022            # mm MeV^-p (0.0022 cm MeV^-p), Bragg-Kleeman for water
BK_P = 1.77


def prior_poly(E_kin: float = 200.0, s_max: float = 200.0, degree: int = 5) -> np.ndarray:
    """Coefficients c_0..c_d (ascending, MeV^-2, depth in mm) of a polynomial
    fit of 1/(beta p)^2 over water depth [0, s_max], from the Bragg-Kleeman
    range-energy relation, least squares in relative error.  This is input
    data for the path prior, fitted once here; both implementations read the
    coefficients."""
    R0 = BK_ALPHA * E_kin ** BK_P
    s = np.linspace(0.0, s_max, 2001)
    E = ((R0 - s) / BK_ALPHA) ** (1.0 / BK_P)
    bp = (E * E + 2.0 * E * M_PROTON) / (E + M_PROTON)
    f = 1.0 / (bp * bp)
    V = np.vander(s / s_max, degree + 1, increasing=True)
    cs, *_ = np.linalg.lstsq(V / f[:, None], np.ones_like(f), rcond=None)
    return cs / s_max ** np.arange(degree + 1)


# ----------------------------------------------------------------- configs
@dataclass
class Config:
    key: int
    name: str
    grid: Grid
    phantom: Phantom
    beam: Beam
    n: int
    seed: int
    perm_seed: int
    algo: str                 # "art" | "drop"
    sweeps: int
    block: int
    lam: float
    rows: str                 # "f32" | "f16" | "fused"
    x0: str = "hull"


def _phantom_tiny() -> Phantom:
    body = Shape(1, (0.0, 0.0, 0.0), (28.0, 28.0, 7.0), 0.0, -7.0, 7.0, 1.0)
    ins = []
    for ang, rsp in zip((0.0, 120.0, 240.0), (0.3, 1.1, 1.6)):
        a = math.radians(ang)
        ins.append(Shape(1, (14.0 * math.cos(a), 14.0 * math.sin(a), 0.0), (6.0, 6.0, 7.0), 0.0, -7.0, 7.0, rsp))
    return Phantom(body, ins)


def _phantom_head(seed: int, n_ins: int = 8) -> Phantom:
    """Elliptic head (a=95, b=80 mm, z in [-18, 18], RSP 1.0) with seeded
    non-overlapping ellipsoidal inserts at least 3 mm inside the body."""
    A, B, Z = 95.0, 80.0, 18.0
    body = Shape(1, (0.0, 0.0, 0.0), (A, B, Z), 0.0, -Z, Z, 1.0)
    rng = np.random.default_rng(seed)
    ins: list[Shape] = []
    tries = 0
    while len(ins) < n_ins:
        tries += 1
        if tries > 100000:
            raise RuntimeError("phantom placement failed")
        ax = float(rng.uniform(6, 20))
        ay = float(rng.uniform(6, 20))
        az = float(rng.uniform(6, 15))
        yaw = float(rng.uniform(0, math.pi))
        r = max(ax, ay)
        cx = float(rng.uniform(-A, A))
        cy = float(rng.uniform(-B, B))
        czmax = Z - 3.0 - az
        cz = float(rng.uniform(-czmax, czmax)) if czmax > 0 else 0.0
        # bounding circle (radius r + 3) must lie inside the body ellipse
        th = np.linspace(0, 2 * np.pi, 90, endpoint=False)
        px = cx + (r + 3.0) * np.cos(th)
        py = cy + (r + 3.0) * np.sin(th)
        if np.any((px / A) ** 2 + (py / B) ** 2 > 1.0):
            continue
        ok = True
        R = max(ax, ay, az)
        for s in ins:
            if math.dist((cx, cy, cz), s.c) < R + max(s.ax) + 2.0:
                ok = False
                break
        if not ok:
            continue
        rsp = float(rng.uniform(0.2, 1.8))
        ins.append(Shape(0, (cx, cy, cz), (ax, ay, az), yaw, cz - az, cz + az, rsp))
    return Phantom(body, ins)


def config(key: int, n: int | None = None) -> Config:
    """The five workloads (1: tiny ART parity case; 2: 1e7 histories with
    cached rows; 3: 2e8 histories, rows recomputed every sweep; 4: config 2
    with FP16 row lengths; 5: learned warm start on config-3 data)."""
    if key == 1:
        g = Grid(64, 64, 16, 1.0, 1.0, 1.0, -32.0, -32.0, -8.0)
        c = Config(1, "tiny", g, _phantom_tiny(), Beam(90, 40.0, 10.0, 5e-3, -55.0, 55.0),
                   100_000, seed=1, perm_seed=101, algo="art", sweeps=10, block=1, lam=0.5, rows="f32")
    elif key in (2, 4):
        g = Grid(200, 200, 40, 1.0, 1.0, 1.0, -100.0, -100.0, -20.0)
        c = Config(key, "head-1e7" if key == 2 else "head-1e7-f16", g, _phantom_head(2),
                   Beam(180, 125.0, 25.0, 5e-3, -150.0, 150.0, step=2.0), 10_000_000, seed=2, perm_seed=202,
                   algo="drop", sweeps=6, block=200_000, lam=0.5, rows="f32" if key == 2 else "f16")
    elif key in (3, 5):
        g = Grid(200, 200, 40, 1.0, 1.0, 1.0, -100.0, -100.0, -20.0)
        c = Config(key, "head-2e8" if key == 3 else "head-2e8-warm", g, _phantom_head(3),
                   Beam(180, 125.0, 25.0, 5e-3, -150.0, 150.0, step=2.0), 200_000_000, seed=3, perm_seed=303,
                   algo="drop", sweeps=8, block=200_000, lam=0.5, rows="fused")
    else:
        raise ValueError(key)
    if n is not None:
        c.n = int(n)
    return c


def training_config(phantom_seed: int, n: int, block: int = 200_000, lam: float = 0.5) -> Config:
    """A head phantom of the config-2/3 family with its own seed (phantom and
    histories both seeded by phantom_seed), for the warm-start network's
    training pairs: same grid, beam, block size and relaxation as the
    workload it is evaluated on, so that its inputs look alike."""
    g = Grid(200, 200, 40, 1.0, 1.0, 1.0, -100.0, -100.0, -20.0)
    return Config(5, f"head-train-{phantom_seed}", g, _phantom_head(phantom_seed),
                  Beam(180, 125.0, 25.0, 5e-3, -150.0, 150.0, step=2.0), int(n), seed=phantom_seed,
                  perm_seed=phantom_seed + 100_000, algo="drop", sweeps=20, block=block, lam=lam, rows="f32")


# ----------------------------------------------------------------- generation
def _params_c(cfg: Config) -> _Params:
    b = cfg.beam
    p = _Params()
    p.n_angles = b.n_angles
    p.t_half = b.t_half
    p.v_half = b.v_half
    p.slope_sigma = b.slope_sigma
    p.u_in = b.u_in
    p.u_out = b.u_out
    p.step = b.step
    p.E_kin = b.E_kin
    p.bk_alpha = BK_ALPHA
    p.bk_p = BK_P
    p.m_p = M_PROTON
    p.E0_hl = E0_HIGHLAND
    p.X0 = X0_WATER
    p.highland_log = 1 if b.highland_log else 0
    p.scatter = 1 if b.scatter else 0
    p.wepl_sigma = b.wepl_sigma
    p.body_rxy = max(cfg.phantom.body.ax[0], cfg.phantom.body.ax[1])
    return p


def generate(cfg: Config, n: int | None = None, start: int = 0, seed: int | None = None,
             threads: int | None = None) -> dict:
    """Histories [start, start+n) of the seeded sequence, as float32 SoA."""
    lib = _load()
    n = cfg.n if n is None else int(n)
    seed = cfg.seed if seed is None else seed
    out = {k: np.empty(n, dtype=np.float32) for k in HIST_FIELDS}
    shapes, ns = cfg.phantom.shapes_c()
    p = _params_c(cfg)
    fp = ctypes.POINTER(ctypes.c_float)
    ptrs = [out[k].ctypes.data_as(fp) for k in HIST_FIELDS]
    fails = lib.pctgen_histories(ctypes.byref(p), shapes, ns, ctypes.c_uint64(seed), start, n, *ptrs,
                                 threads or default_threads())
    if fails:
        raise RuntimeError(f"{fails} histories could not be generated")
    return out


def generate_misses(cfg: Config, n: int, start: int = 0, seed: int | None = None,
                    threads: int | None = None) -> dict:
    """Histories [start, start+n) of the seeded stream of protons that miss
    the body (straight lines through air, WEPL = noise), float32 SoA: the
    input of the space-carving hull."""
    lib = _load()
    n = int(n)
    seed = cfg.seed if seed is None else seed
    out = {k: np.empty(n, dtype=np.float32) for k in HIST_FIELDS}
    shapes, ns = cfg.phantom.shapes_c()
    p = _params_c(cfg)
    fp = ctypes.POINTER(ctypes.c_float)
    ptrs = [out[k].ctypes.data_as(fp) for k in HIST_FIELDS]
    fails = lib.pctgen_miss_histories(ctypes.byref(p), shapes, ns, ctypes.c_uint64(seed), start, n, *ptrs,
                                      threads or default_threads())
    if fails:
        raise RuntimeError(f"{fails} miss histories could not be generated")
    return out


_lib_gpu = None


def _load_gpu():
    global _lib_gpu
    if _lib_gpu is None:
        if not os.path.exists(_SO_GPU):
            raise ImportError(f"{_SO_GPU} is missing: run synth.build()")
        lib = ctypes.CDLL(_SO_GPU)
        lib.pctgen_gpu_histories.restype = ctypes.c_int
        lib.pctgen_gpu_histories.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64,
                                             ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p),
                                             ctypes.c_void_p, ctypes.c_void_p]
        _lib_gpu = lib
    return _lib_gpu


def generate_gpu(cfg: Config, n: int | None = None, start: int = 0, seed: int | None = None, device=None) -> dict:
    """Histories [start, start+n) of the same seeded sequence as generate(),
    made on the GPU straight into device memory: a dict of float32 torch
    tensors (torch supplies the allocations and the stream)."""
    import torch
    lib = _load_gpu()
    n = cfg.n if n is None else int(n)
    seed = cfg.seed if seed is None else seed
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    out = {k: torch.empty(n, dtype=torch.float32, device=dev) for k in HIST_FIELDS}
    fails = torch.zeros(1, dtype=torch.int64, device=dev)
    shapes, ns = cfg.phantom.shapes_c()
    p = _params_c(cfg)
    ptrs = (ctypes.c_void_p * 10)(*[out[k].data_ptr() for k in HIST_FIELDS])
    stream = torch.cuda.current_stream(dev).cuda_stream
    rc = lib.pctgen_gpu_histories(ctypes.addressof(p), ctypes.addressof(shapes), ns, ctypes.c_uint64(seed), start, n,
                                  ptrs, fails.data_ptr(), stream)
    if rc != 0:
        raise RuntimeError(f"device history generation failed ({rc})")
    nf = int(fails.item())
    if nf:
        raise RuntimeError(f"{nf} histories could not be generated")
    return out


def block_order(n: int, seed: int) -> np.ndarray:
    """Seeded Fisher-Yates permutation (splitmix64 draws): consecutive slices
    of it form the blocks of the block-iterative solver."""
    lib = _load()
    out = np.empty(n, dtype=np.int64)
    lib.pctgen_permutation(n, ctypes.c_uint64(seed), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def segment_wepl(ph: Phantom, P, Q) -> float:
    lib = _load()
    shapes, ns = ph.shapes_c()
    a = (ctypes.c_double * 3)(*P)
    b = (ctypes.c_double * 3)(*Q)
    return lib.pctgen_segment_wepl(shapes, ns, a, b)


def point_rsp(ph: Phantom, X) -> float:
    lib = _load()
    shapes, ns = ph.shapes_c()
    return lib.pctgen_point_rsp(shapes, ns, (ctypes.c_double * 3)(*X))


def truth_image(cfg: Config, ss: int = 4, threads: int | None = None) -> np.ndarray:
    lib = _load()
    g = cfg.grid
    out = np.empty(g.M, dtype=np.float32)
    shapes, ns = cfg.phantom.shapes_c()
    lib.pctgen_truth_image(shapes, ns, g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz, ss,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), threads or default_threads())
    return out


def hull_mask(cfg: Config) -> np.ndarray:
    """1 for voxels whose centre lies in the body (the reconstruction hull)."""
    g = cfg.grid
    b = cfg.phantom.body
    X, Y, Z = g.centers()
    inside = ((X / b.ax[0]) ** 2 + (Y / b.ax[1]) ** 2 <= 1.0) & (Z >= b.z0) & (Z <= b.z1)
    return inside.astype(np.uint8)


def roi_labels(cfg: Config, erode_vox: float = 2.0) -> np.ndarray:
    """Label k (1-based) for voxels inside insert k eroded by erode_vox voxels
    (the ROI analysis of Sec. 3.2 / 4.2: ROIs kept away from walls and ends)."""
    g = cfg.grid
    X, Y, Z = g.centers()
    lab = np.zeros(g.M, dtype=np.uint8)
    e = erode_vox * min(g.dx, g.dy, g.dz)
    body = cfg.phantom.body
    for n, s in enumerate(cfg.phantom.inserts, start=1):
        cs, sn = math.cos(s.yaw), math.sin(s.yaw)
        px, py = X - s.c[0], Y - s.c[1]
        lx, ly = cs * px + sn * py, -sn * px + cs * py
        ax, ay = s.ax[0] - e, s.ax[1] - e
        if ax <= 0 or ay <= 0:
            continue
        if s.kind == 0:
            az = s.ax[2] - e
            if az <= 0:
                continue
            m = (lx / ax) ** 2 + (ly / ay) ** 2 + ((Z - s.c[2]) / az) ** 2 <= 1.0
        else:
            m = ((lx / ax) ** 2 + (ly / ay) ** 2 <= 1.0) & (Z >= s.z0 + e) & (Z <= s.z1 - e)
        # keep away from the phantom caps too
        m &= (Z >= body.z0 + e) & (Z <= body.z1 - e)
        lab[m] = n
    return lab


def insert_rsp(cfg: Config) -> np.ndarray:
    return np.array([s.rsp for s in cfg.phantom.inserts], dtype=np.float64)
