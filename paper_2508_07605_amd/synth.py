"""Seeded synthetic workloads for the CF-completion hot path.

The paper's matrices come from profiling real applications under CPU x GPU power caps
(Section III-A.3, Eq. 1; Section III-B.2: a few profiled entries per new application).
Those traces are not available, so every input here is synthetic, with the shape of the
paper's normalized-performance matrices: value 1 at the no-cap setting, values in
roughly [0.4, 1], multiplicative CPU and GPU sensitivity per application.

This module only draws data: cap grids, per-application sensitivity parameters, the
noiseless truth, observation sets, noisy observed values, random initial factors and
network weights.  It contains no step of the completion method itself.  Both the oracle
and the GPU path receive what it returns as plain arrays.

Streams: numpy PCG64 seeded as ``default_rng([cfg_id, stream, seed, 20250811])``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_TAG = 20250811

# independent random streams per configuration
S_APPS, S_COUNTS, S_SETS, S_NOISE, S_INIT, S_MLP, S_REF, S_EVAL, S_POWER, S_COUNTERS, S_PRED, S_NCF = range(12)


def rng(cfg_id: int, stream: int, seed: int = 0) -> np.random.Generator:
    return np.random.default_rng([cfg_id, stream, seed, SEED_TAG])


# ----------------------------------------------------------------------------- grid
@dataclasses.dataclass
class Grid:
    """Setting grid C x G, flattened CPU-major: s = a * n_gpu + b."""
    n_cpu: int
    n_gpu: int
    cpu_w: np.ndarray  # f64[n] CPU cap (W) of setting s
    gpu_w: np.ndarray  # f64[n] GPU cap (W) of setting s
    base: int          # index of the no-cap baseline (C_max, G_max)

    @property
    def n(self) -> int:
        return self.n_cpu * self.n_gpu


def cap_grid(n_cpu: int, n_gpu: int, cpu_lo=120.0, cpu_hi=270.0, gpu_lo=100.0, gpu_hi=250.0) -> Grid:
    """Evenly spaced caps.  The paper never lists its watt values; only the ratios to the
    maximum enter the truth and only c + g enters the selection rule (Alg. 2)."""
    c = np.linspace(cpu_lo, cpu_hi, n_cpu)
    g = np.linspace(gpu_lo, gpu_hi, n_gpu)
    cpu_w = np.repeat(c, n_gpu)
    gpu_w = np.tile(g, n_cpu)
    return Grid(n_cpu, n_gpu, cpu_w, gpu_w, n_cpu * n_gpu - 1)


# ----------------------------------------------------------------------------- apps
@dataclasses.dataclass
class Apps:
    beta: np.ndarray   # CPU share of the runtime, Beta(2, 2)
    gc: np.ndarray     # CPU cap sensitivity exponent, U(0.3, 1.0)
    gg: np.ndarray     # GPU cap sensitivity exponent, U(0.3, 1.0)

    def __len__(self):
        return len(self.beta)

    def take(self, rows) -> "Apps":
        return Apps(self.beta[rows], self.gc[rows], self.gg[rows])


def draw_apps(r: np.random.Generator, m: int) -> Apps:
    return Apps(r.beta(2.0, 2.0, m), r.uniform(0.3, 1.0, m), r.uniform(0.3, 1.0, m))


def truth_at(apps: Apps, grid: Grid, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Noiseless normalized performance t_is = 1 / (beta (Cmax/c)^gc + (1-beta) (Gmax/g)^gg)
    at index pairs (rows[t], cols[t]); f64."""
    cmax = grid.cpu_w.max()
    gmax = grid.gpu_w.max()
    b = apps.beta[rows]
    slow = b * (cmax / grid.cpu_w[cols]) ** apps.gc[rows] + (1.0 - b) * (gmax / grid.gpu_w[cols]) ** apps.gg[rows]
    return 1.0 / slow


def truth_dense(apps: Apps, grid: Grid) -> np.ndarray:
    """Full truth block, f64[len(apps), n]."""
    m = len(apps)
    rows = np.repeat(np.arange(m), grid.n)
    cols = np.tile(np.arange(grid.n), m)
    return truth_at(apps, grid, rows, cols).reshape(m, grid.n)


# ----------------------------------------------------------------------------- observation sets
def draw_counts(r: np.random.Generator, m: int, n: int, spec) -> np.ndarray:
    """Observed entries per row.  spec: ("full",) | ("fixed", c) | ("uniform", lo, hi) |
    ("zipf", a, lo, hi) = truncated pmf proportional to c^-a on [lo, hi]."""
    kind = spec[0]
    if kind == "full":
        return np.full(m, n, dtype=np.int64)
    if kind == "fixed":
        return np.full(m, int(spec[1]), dtype=np.int64)
    if kind == "uniform":
        return r.integers(int(spec[1]), int(spec[2]) + 1, size=m).astype(np.int64)
    if kind == "zipf":
        a, lo, hi = float(spec[1]), int(spec[2]), int(spec[3])
        ks = np.arange(lo, hi + 1)
        p = ks.astype(np.float64) ** (-a)
        p /= p.sum()
        return r.choice(ks, size=m, p=p).astype(np.int64)
    raise ValueError(spec)


def _sets_by_keys(r: np.random.Generator, counts: np.ndarray, n: int):
    """Uniform c-subsets of [0, n) by random keys: the c smallest of n iid keys per row."""
    m = len(counts)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    chunk = max(1, (1 << 24) // n)
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        c = counts[s:e]
        cmax = int(c.max()) if e > s else 0
        if cmax == 0:
            continue
        keys = r.random((e - s, n))
        if cmax < n:
            part = np.argpartition(keys, cmax - 1, axis=1)[:, :cmax]
        else:
            part = np.broadcast_to(np.arange(n), (e - s, n)).copy()
        # order the candidate block by key: the first c of them are a uniform c-subset
        order = np.argsort(np.take_along_axis(keys, part, axis=1), axis=1)
        part = np.take_along_axis(part, order, axis=1)
        keep = np.arange(cmax)[None, :] < c[:, None]
        part = np.sort(np.where(keep, part, n), axis=1)
        col[row_ptr[s]:row_ptr[e]] = part[keep].astype(np.int32)
    return row_ptr, col


def _sets_by_draws(r: np.random.Generator, counts: np.ndarray, n: int):
    """Uniform c-subsets of [0, n) for rows with c much smaller than n: iid uniform draws
    (2c + 16 per row), keeping the first c distinct values in draw order, which is sampling
    without replacement.  Returns (sorted columns per row as CSR pieces, rows that drew fewer
    than c distinct values)."""
    m = len(counts)
    over = 2 * counts + 16
    optr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(over, out=optr[1:])
    rid = np.repeat(np.arange(m, dtype=np.int64), over)
    key = rid * n + r.integers(0, n, size=int(optr[-1]))
    order = np.argsort(key, kind="stable")  # equal keys stay in draw order
    ks = key[order]
    new = np.ones(len(ks), dtype=bool)
    new[1:] = ks[1:] != ks[:-1]
    first = np.zeros(len(key), dtype=bool)
    first[order[new]] = True
    rank = np.cumsum(first) - 1
    rank -= np.repeat(np.concatenate([[0], np.cumsum(first)[optr[1:-1] - 1]]) if m > 1 else np.zeros(1, np.int64),
                      over)
    keep = first & (rank < np.repeat(counts, over))
    got = np.bincount(rid[keep], minlength=m)
    ks_keep = ks[keep[order]]  # kept keys, already sorted (row-major, then column)
    return ks_keep, got


def draw_sets(r: np.random.Generator, counts: np.ndarray, n: int):
    """Uniform subsets without replacement, sorted within each row.
    Returns CSR (row_ptr int64[m+1], col int32[nnz]).  Grids of 1024 or more settings draw
    the sparse rows (c <= n / 4) by iid draws with rejection of repeats, the rest by keys."""
    if n < 1024:
        return _sets_by_keys(r, counts, n)
    m = len(counts)
    counts = np.asarray(counts, dtype=np.int64)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    sparse = counts <= n // 4
    chunk = 200_000
    redo = [np.nonzero(~sparse)[0]]
    sp_idx = np.nonzero(sparse)[0]
    for s in range(0, len(sp_idx), chunk):
        ids = sp_idx[s:s + chunk]
        ks, got = _sets_by_draws(r, counts[ids], n)
        ok = got == counts[ids]
        rows_of = ks // n
        good = ok[rows_of]
        kcol = (ks[good] % n).astype(np.int32)
        # scatter the complete rows to their CSR ranges (rows stay in order within the chunk)
        okids = ids[ok]
        dst = np.repeat(row_ptr[okids], counts[okids]) + (
            np.arange(int(counts[okids].sum())) - np.repeat(np.cumsum(counts[okids]) - counts[okids], counts[okids]))
        col[dst] = kcol
        redo.append(ids[~ok])
    redo = np.sort(np.concatenate(redo))
    if len(redo):
        rp, c2 = _sets_by_keys(r, counts[redo], n)
        dst = np.repeat(row_ptr[redo], counts[redo]) + (np.arange(int(rp[-1])) - np.repeat(rp[:-1], counts[redo]))
        col[dst] = c2
    return row_ptr, col


@dataclasses.dataclass
class Rows:
    """A block of application rows in CSR form."""
    apps: Apps
    row_ptr: np.ndarray  # int64[m+1]
    col: np.ndarray      # int32[nnz], sorted and unique within a row
    val: np.ndarray      # float32[nnz], observed normalized performance

    @property
    def m(self) -> int:
        return len(self.row_ptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def counts(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def row_ids(self) -> np.ndarray:
        return np.repeat(np.arange(self.m, dtype=np.int64), self.counts())


def draw_rows(cfg_id: int, grid: Grid, m: int, count_spec, seed: int = 0, noise: float = 0.02) -> Rows:
    apps = draw_apps(rng(cfg_id, S_APPS, seed), m)
    counts = draw_counts(rng(cfg_id, S_COUNTS, seed), m, grid.n, count_spec)
    row_ptr, col = draw_sets(rng(cfg_id, S_SETS, seed), counts, grid.n)
    rows = np.repeat(np.arange(m, dtype=np.int64), counts)
    t = truth_at(apps, grid, rows, col.astype(np.int64))
    eps = rng(cfg_id, S_NOISE, seed).standard_normal(len(t))
    val = (t * (1.0 + noise * eps)).astype(np.float32)
    return Rows(apps, row_ptr, col, val)


# ----------------------------------------------------------------------------- factors
def init_factors(cfg_id: int, m: int, n: int, k: int, std: float = 0.1, seed: int = 0):
    """Initial U0 (m x k) and V0 (n x k), iid N(0, std^2), float32."""
    r = rng(cfg_id, S_INIT, seed)
    U0 = (std * r.standard_normal((m, k))).astype(np.float32)
    V0 = (std * r.standard_normal((n, k))).astype(np.float32)
    return U0, V0


def setting_factors(cfg_id: int, grid: Grid, k: int, m_ref: int = 4096, seed: int = 0) -> np.ndarray:
    """Fixed setting factors V (n x k, float32) for fold-in workloads: the balanced rank-k
    truncated SVD of a fully profiled, noiseless reference population of m_ref apps
    (stand-in for the dense offline matrix of Eq. 1).  Balanced means
    V = V_k S_k^(1/2) (n/m_ref)^(1/4), so typical row norms of both factors agree."""
    apps = draw_apps(rng(cfg_id, S_REF, seed), m_ref)
    R = truth_dense(apps, grid)
    _, s, vt = np.linalg.svd(R, full_matrices=False)
    V = vt[:k].T * np.sqrt(s[:k])[None, :] * (grid.n / m_ref) ** 0.25
    return np.ascontiguousarray(V.astype(np.float32))


def mlp_init(cfg_id: int, dims, seed: int = 0):
    """Uniform(+-1/sqrt(fan_in)) weights and biases for a stack of dense layers.
    dims = (d0, d1, ..., dL); layer l maps d_l -> d_{l+1}; W_l has shape (d_{l+1}, d_l).
    Returns a flat list [W0, b0, W1, b1, ...] of float32 arrays."""
    r = rng(cfg_id, S_MLP, seed)
    out = []
    for din, dout in zip(dims[:-1], dims[1:]):
        bound = 1.0 / np.sqrt(din)
        out.append(r.uniform(-bound, bound, (dout, din)).astype(np.float32))
        out.append(r.uniform(-bound, bound, dout).astype(np.float32))
    return out


# ----------------------------------------------------------------------------- configurations
CONFIGS = {
    # 64 dense offline apps + 16 online apps with 6 observed entries; 12 x 10 caps; rank 8
    "tiny": dict(cfg_id=1, n_cpu=12, n_gpu=10, k=8, lam=0.05, sweeps=20, m_dense=64, m_new=16, new_obs=6),
    # 200k apps x 480 settings, truncated Zipf(1.2) on [3, 480] observed counts, rank 32
    "fit": dict(cfg_id=2, n_cpu=24, n_gpu=20, k=32, lam=0.05, sweeps=15, m=200_000, counts=("zipf", 1.2, 3, 480)),
    # same, exponent tuned so the density is 5 %
    "fit_d5": dict(cfg_id=6, n_cpu=24, n_gpu=20, k=32, lam=0.05, sweeps=15, m=200_000,
                   counts=("zipf", 1.6824, 3, 480)),
    # 1M new apps with 4..24 observed settings each against fixed 480 x 32 setting factors; the
    # fold-in of a new row is the plain ridge solution (lambda I, weighted=False)
    "foldin": dict(cfg_id=3, n_cpu=24, n_gpu=20, k=32, lam=0.05, weighted=False, m=1_000_000,
                   counts=("uniform", 4, 24)),
    # surrogate 960 -> 256 -> 256 -> 32 trained for 10 epochs on 2M fold-ins of the same generator
    # (other seed)
    "surrogate": dict(cfg_id=3, n_cpu=24, n_gpu=20, k=32, lam=0.05, weighted=False, m_train=2_000_000, train_seed=1,
                      hidden=256, batch=4096, lr=1e-3, epochs=10, tau=0.02, counts=("uniform", 4, 24)),
    # 2M apps x 1920 settings, ~2 % density, rank 64
    "large": dict(cfg_id=5, n_cpu=48, n_gpu=40, k=64, lam=0.05, sweeps=10, m=2_000_000,
                  counts=("zipf", 1.6931, 3, 1920), gamma=0.05, batch=16384, hidden=256),
}


def grid_of(name: str) -> Grid:
    c = CONFIGS[name]
    return cap_grid(c["n_cpu"], c["n_gpu"])


def tiny_problem(seed: int = 0):
    """The tiny configuration: dense offline block, sparse online block and their union."""
    c = CONFIGS["tiny"]
    grid = grid_of("tiny")
    dense = draw_rows(c["cfg_id"], grid, c["m_dense"], ("full",), seed=seed)
    new = draw_rows(c["cfg_id"], grid, c["m_new"], ("fixed", c["new_obs"]), seed=seed + 1000)
    rp = np.concatenate([dense.row_ptr, dense.row_ptr[-1] + new.row_ptr[1:]])
    union = Rows(Apps(np.concatenate([dense.apps.beta, new.apps.beta]),
                      np.concatenate([dense.apps.gc, new.apps.gc]),
                      np.concatenate([dense.apps.gg, new.apps.gg])),
                 rp, np.concatenate([dense.col, new.col]), np.concatenate([dense.val, new.val]))
    return grid, dense, new, union


def latent_rows(cfg_id: int, grid: Grid, V: np.ndarray, m: int, seed: int = 0, n_proto: int = 4096,
                noise: float = 0.01) -> np.ndarray:
    """Application factors (m x k, float32) whose predictions u . v_s look like normalized
    performance: n_proto prototype apps are projected (least squares) from their noiseless
    truth rows onto the setting factors V, and every row is a prototype plus N(0, noise^2)."""
    apps = draw_apps(rng(cfg_id, S_EVAL, seed), n_proto)
    T = truth_dense(apps, grid)
    Vd = V.astype(np.float64)
    proto = np.linalg.lstsq(Vd, T.T, rcond=None)[0].T  # n_proto x k
    r = rng(cfg_id, S_EVAL, seed + 1)
    pick = r.integers(0, n_proto, size=m)
    U = proto[pick] + noise * r.standard_normal((m, V.shape[1]))
    return np.ascontiguousarray(U.astype(np.float32))


# ----------------------------------------------------------------------------- power traces
def power_traces(cfg_id: int, T: int, L: int, seed: int = 0, p_never: float = 0.1,
                 p_dip: float = 0.01) -> np.ndarray:
    """GPU power readings (W), T traces x L samples, float32: a CPU-side phase of random length
    at 25-55 W, then a GPU phase at 120-280 W with rare dips to 20-59 W (data loading, sync);
    a fraction p_never of the traces stays in the CPU phase.  Stand-in for the paper's power
    patterns of applications with long CPU phases (Fig. 5)."""
    r = rng(cfg_id, S_POWER, seed)
    start = r.integers(0, L, size=T)
    start[r.random(T) < p_never] = L
    lo = r.uniform(25.0, 55.0, size=(T, 1))
    hi = r.uniform(120.0, 280.0, size=(T, 1))
    t = np.arange(L)[None, :]
    gpu = t >= start[:, None]
    p = np.where(gpu, hi, lo) + r.normal(0.0, 3.0, size=(T, L))
    dip = gpu & (r.random((T, L)) < p_dip)
    p = np.where(dip, r.uniform(20.0, 59.0, size=(T, L)), p)
    return np.ascontiguousarray(p.astype(np.float32))


# ----------------------------------------------------------------------------- offline predictor
# Feature ranges of a profiled run besides the two caps (uniform draws): memory throughput
# (GB/s), instructions per second, SM clock (MHz), DRAM active rate, FP active rate.
COUNTER_RANGES = ((50.0, 1500.0), (1.0e9, 5.0e10), (800.0, 1410.0), (0.0, 1.0), (0.0, 1.0))


def run_features(cfg_id: int, grid: Grid, setting: np.ndarray, seed: int = 0) -> np.ndarray:
    """Seven features per profiled run (float32 [runs, 7]): the CPU and GPU caps of the run's
    setting, then synthetic counter readings (COUNTER_RANGES).  Stand-in for the counters the
    paper collects online (Table I); no real counter data is available."""
    r = rng(cfg_id, S_COUNTERS, seed)
    setting = np.asarray(setting, dtype=np.int64)
    X = np.empty((len(setting), 7), dtype=np.float32)
    X[:, 0] = grid.cpu_w[setting]
    X[:, 1] = grid.gpu_w[setting]
    for f, (lo, hi) in enumerate(COUNTER_RANGES):
        X[:, 2 + f] = r.uniform(lo, hi, size=len(setting))
    return X


def predictor_params(cfg_id: int, grid: Grid, seed: int = 0, hidden: int = 64) -> dict:
    """Random weights of the 7 -> 64 -> 64 -> 1 predictor (He-uniform hidden layers, small
    output layer, output bias 0.75) and the centring/scaling of each feature from the mean and
    standard deviation of the ranges it is drawn from.  No trained weights exist."""
    r = rng(cfg_id, S_PRED, seed)
    ranges = [(grid.cpu_w.min(), grid.cpu_w.max()), (grid.gpu_w.min(), grid.gpu_w.max())] + list(COUNTER_RANGES)
    mu = np.array([(lo + hi) / 2 for lo, hi in ranges])
    sd = np.array([(hi - lo) / np.sqrt(12.0) for lo, hi in ranges])
    b1w, b2w = np.sqrt(6.0 / 7), np.sqrt(6.0 / hidden)
    p = dict(mu=mu, rs=1.0 / sd,
             W1=r.uniform(-b1w, b1w, (hidden, 7)), b1=r.uniform(-0.1, 0.1, hidden),
             W2=r.uniform(-b2w, b2w, (hidden, hidden)), b2=r.uniform(-0.1, 0.1, hidden),
             w3=r.uniform(-0.05, 0.05, hidden), b3=np.array([0.75]))
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in p.items()}


# ----------------------------------------------------------------------------- NCF
NCF = dict(d=32, hidden=64, steps=30, eta=0.5, mu=1e-3)


def ncf_params(cfg_id: int, n: int, seed: int = 0, d: int = 32, hidden: int = 64) -> dict:
    """Random NCF weights (no trained model exists): setting embeddings S (n x d) ~ N(0, 1),
    LeCun-normal hidden layers (std 1/sqrt(fan_in), the SELU initialisation), zero hidden
    biases, output weights ~ N(0, 1/hidden) and output bias 0.75 (the middle of the normalized
    performance range)."""
    r = rng(cfg_id, S_NCF, seed)
    p = dict(S=r.standard_normal((n, d)),
             W1=r.standard_normal((hidden, 2 * d)) / np.sqrt(2 * d), b1=np.zeros(hidden),
             W2=r.standard_normal((hidden, hidden)) / np.sqrt(hidden), b2=np.zeros(hidden),
             w3=r.standard_normal(hidden) / np.sqrt(hidden), b3=np.array([0.75]))
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in p.items()}
