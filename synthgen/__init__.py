"""Seeded synthetic inputs for the randomized (H-)Tucker path.

This module only *draws* inputs: low-rank-plus-noise tensors, fiber index
sets and Gaussian sketch matrices.  It holds none of the decomposition's
arithmetic (no sketch, QR, truncation, core or error computation), so both
the FP64 oracle and the GPU path can consume the same bytes without sharing
any code of the method.

Every random quantity the method itself would draw (the fiber indices of
the sampling matrix E_k and the Gaussian Omega_k, Alg. 1 and Alg. 2 of the
paper) is generated here on the host and passed in as an input.

Storage dtypes: "f64", "f32", "f16" map to the numpy types of the same
name; "bf16" is stored as ``uint16`` holding the upper half of the IEEE
binary32 pattern (round-to-nearest-even).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2603_21379

# purposes for SeedSequence keys
_CORE, _FACTORS, _NOISE, _SKETCH, _BATCH, _TRANSFER = range(6)

DTYPES = ("f64", "f32", "bf16", "f16")


def _ss(cfg: int, purpose: int, *sub: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([SEED_BASE, int(cfg), int(purpose), *[int(s) for s in sub]])


def _rng(cfg: int, purpose: int, *sub: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(_ss(cfg, purpose, *sub)))


# ---------------------------------------------------------------- storage dtypes
def to_storage(x: np.ndarray, dtype: str) -> np.ndarray:
    """Round a float64/float32 array to the storage dtype (RNE)."""
    if dtype == "f64":
        return np.ascontiguousarray(x, dtype=np.float64)
    if dtype == "f32":
        return np.ascontiguousarray(x, dtype=np.float32)
    if dtype == "f16":
        return np.ascontiguousarray(x, dtype=np.float16)
    if dtype == "bf16":
        u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
        rounded = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) >> np.uint32(16)
        return rounded.astype(np.uint16)
    raise ValueError(f"unknown dtype {dtype}")


def to_f64(x: np.ndarray, dtype: str) -> np.ndarray:
    """Exact upcast of stored values to float64."""
    if dtype == "bf16":
        return (x.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    return np.asarray(x, dtype=np.float64)


def itemsize(dtype: str) -> int:
    return {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[dtype]


def factor_dtype(dtype: str) -> str:
    """dtype of factors / core for a given tensor storage dtype."""
    return "f64" if dtype == "f64" else "f32"


# ---------------------------------------------------------------- primitives
def haar(n: int, r: int, rng: np.random.Generator) -> np.ndarray:
    """n x r matrix with orthonormal columns, Haar distributed."""
    a = rng.standard_normal((n, r))
    q, rr = np.linalg.qr(a)
    s = np.sign(np.diag(rr))
    s[s == 0] = 1.0
    return q * s


def decay_core(ranks, decay: float, rng: np.random.Generator) -> np.ndarray:
    """Gaussian core scaled by prod_k decay**i_k (0-based indices)."""
    g = rng.standard_normal(tuple(ranks))
    for k, r in enumerate(ranks):
        shape = [1] * len(ranks)
        shape[k] = r
        g = g * (float(decay) ** np.arange(r, dtype=np.float64)).reshape(shape)
    return g


def _threads() -> int:
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _single_blas(fn):
    """Run a generator with one BLAS thread.

    A multi-threaded BLAS may split a product differently from run to run
    (or with the thread count), which changes the last bits of the result;
    the generators parallelise over slabs themselves instead, so the same
    seed gives the same bytes on every run."""
    import functools

    @functools.wraps(fn)
    def wrapped(*a, **kw):
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1, user_api="blas"):
            return fn(*a, **kw)
    return wrapped


def _parallel_slabs(fn, count: int, threads: int | None):
    with ThreadPoolExecutor(threads or _threads()) as ex:
        list(ex.map(fn, range(count)))


# ---------------------------------------------------------------- Tucker tensors
@dataclass
class TuckerInput:
    dims: tuple
    ranks: tuple
    dtype: str
    X: np.ndarray            # storage dtype, C-order
    core: np.ndarray         # generating core (f64)
    factors: list            # generating orthonormal factors (f64)
    scale: float             # X_sig = scale * (core x_k factors)
    noise: float             # relative noise level


@_single_blas
def tucker_tensor(dims, ranks, decay: float, noise: float, cfg: int, dtype: str = "f64",
                  run: int = 0, threads: int | None = None) -> TuckerInput:
    """Low-rank Tucker tensor plus relative Gaussian noise.

    X = X_sig / rms(X_sig) + noise * N(0,1); the signal has orthonormal
    factors, so rms(X_sig) = ||core||_F / sqrt(prod dims).  Built slab by slab
    along mode 0 (one slab per index of mode 0, each with its own child seed
    for the noise), so the result does not depend on the thread count.
    """
    dims = tuple(int(n) for n in dims)
    ranks = tuple(int(r) for r in ranks)
    d = len(dims)
    core = decay_core(ranks, decay, _rng(cfg, _CORE, run))
    frng = _rng(cfg, _FACTORS, run)
    factors = [haar(n, r, frng) for n, r in zip(dims, ranks)]
    N = math.prod(dims)
    scale = math.sqrt(N) / float(np.linalg.norm(core))
    X = np.empty(dims, dtype={"f64": np.float64, "f32": np.float32, "f16": np.float16,
                              "bf16": np.uint16}[dtype])
    # core contracted with nothing yet; per slab: core x_0 U0[i0] x_k U_k
    core_s = core * scale

    def slab(i0: int):
        t = np.tensordot(factors[0][i0], core_s, axes=(0, 0))        # (r1..r_{d-1})
        t = t[None]
        for k in range(1, d):
            t = np.tensordot(t, factors[k], axes=([1], [1]))           # appends n_k
        t = t[0]
        if noise:
            g = _rng(cfg, _NOISE, run, i0)
            t = t + noise * g.standard_normal(t.shape)
        X[i0] = to_storage(t, dtype)

    _parallel_slabs(slab, dims[0], threads)
    return TuckerInput(dims, ranks, dtype, X, core, factors, scale, noise)


# ---------------------------------------------------------------- sketch operands
@dataclass
class Sketch:
    """Fiber sample of one mode (or tree node) and its Gaussian test matrix."""
    idx: np.ndarray   # int64 [s], strictly increasing column indices of the unfolding
    omega: np.ndarray  # [s, ell], values already rounded to omega_dtype, stored float64
    omega_dtype: str

    @property
    def s(self):
        return int(self.idx.shape[0])

    @property
    def ell(self):
        return int(self.omega.shape[1])


def sample_columns(ncols: int, s: int, rng: np.random.Generator) -> np.ndarray:
    """s distinct column indices of [0, ncols), uniform without repetition, sorted."""
    if s > ncols:
        raise ValueError("cannot sample more columns than exist")
    if s == ncols:
        return np.arange(ncols, dtype=np.int64)
    idx = rng.choice(ncols, size=s, replace=False, shuffle=False)
    return np.sort(idx.astype(np.int64))


def gaussian(s: int, ell: int, rng: np.random.Generator, omega_dtype: str) -> np.ndarray:
    om = rng.standard_normal((s, ell))
    return to_f64(to_storage(om, omega_dtype), omega_dtype)


def mode_sketches(dims, ells, ss, cfg: int, omega_dtype: str, run: int = 0, dense=False):
    """One Sketch per mode: s_k sampled mode-k fibers and Omega_k (s_k x ell_k)."""
    dims = tuple(int(n) for n in dims)
    N = math.prod(dims)
    out = []
    for k, n in enumerate(dims):
        ncols = N // n
        s = ncols if dense else int(ss[k])
        rng = _rng(cfg, _SKETCH, run, k)
        idx = sample_columns(ncols, s, rng)
        out.append(Sketch(idx, gaussian(s, int(ells[k]), rng, omega_dtype), omega_dtype))
    return out


def default_s(dims, alpha: int = 10):
    """s_k = min(alpha * n_k, n_{!=k}), the rule of thumb s_k >= 10 n_k."""
    N = math.prod(dims)
    return [min(alpha * n, N // n) for n in dims]


def default_ell(dims, ranks, p: int):
    N = math.prod(dims)
    return [min(r + p, n, N // n) for n, r in zip(dims, ranks)]


# ---------------------------------------------------------------- dimension trees
@dataclass
class DimTree:
    """Balanced binary dimension tree in heap order (node 0 = root).

    Node t covers the modes first[t] .. first[t]+count[t]-1; its left child
    takes the first ceil(count/2) of them.  left/right are -1 for leaves.
    """
    order: int
    first: list = field(default_factory=list)
    count: list = field(default_factory=list)
    left: list = field(default_factory=list)
    right: list = field(default_factory=list)
    level: list = field(default_factory=list)

    @property
    def num_nodes(self):
        return len(self.first)

    def is_leaf(self, t):
        return self.left[t] < 0

    def modes(self, t):
        return list(range(self.first[t], self.first[t] + self.count[t]))

    def leaf_of_mode(self, k):
        for t in range(self.num_nodes):
            if self.is_leaf(t) and self.first[t] == k:
                return t
        raise KeyError(k)


def balanced_tree(order: int) -> DimTree:
    """Heap-indexed balanced tree; left child = first ceil(|S|/2) modes of S."""
    if order < 2:
        raise ValueError("a dimension tree needs order >= 2")
    tr = DimTree(order)
    queue = [(0, order, 0)]
    # breadth-first construction gives heap indices level by level
    while queue:
        nxt = []
        for first, count, lev in queue:
            tr.first.append(first)
            tr.count.append(count)
            tr.level.append(lev)
            tr.left.append(-1)
            tr.right.append(-1)
        base = len(tr.first) - len(queue)
        for j, (first, count, lev) in enumerate(queue):
            if count > 1:
                cl = (count + 1) // 2
                tr.left[base + j] = base + len(queue) + len(nxt)
                nxt.append((first, cl, lev + 1))
                tr.right[base + j] = base + len(queue) + len(nxt)
                nxt.append((first + cl, count - cl, lev + 1))
        queue = nxt
    return tr


@dataclass
class HTInput:
    dims: tuple
    X: np.ndarray
    dtype: str
    tree: DimTree
    leaf_bases: dict    # node -> n_k x r orthonormal
    transfers: dict     # internal non-root node -> (r, r_l, r_r)
    root: np.ndarray    # (1, r_l, r_r)
    scale: float
    noise: float


@_single_blas
def ht_tensor(n: int, order: int, rank: int, noise: float, cfg: int, dtype: str = "f32",
              run: int = 0, threads: int | None = None) -> HTInput:
    """Tensor of hierarchical rank `rank` on the balanced tree, plus noise.

    Leaves get Haar bases, internal non-root nodes a Gaussian transfer tensor
    whose mode-1 unfolding has orthonormal rows (so every nested basis is
    orthonormal), the root a Gaussian 1 x r x r tensor.
    """
    tr = balanced_tree(order)
    rng = _rng(cfg, _TRANSFER, run)
    leaf, trans = {}, {}
    for t in range(tr.num_nodes):
        if tr.is_leaf(t):
            leaf[t] = haar(n, min(rank, n), rng)
    rank_of = {}

    def rk(t):
        if t in rank_of:
            return rank_of[t]
        if tr.is_leaf(t):
            rank_of[t] = leaf[t].shape[1]
        else:
            rank_of[t] = min(rank, rk(tr.left[t]) * rk(tr.right[t]))
        return rank_of[t]

    for t in range(1, tr.num_nodes):
        if not tr.is_leaf(t):
            rl, rr, r = rk(tr.left[t]), rk(tr.right[t]), rk(t)
            b1t = haar(rl * rr, r, rng)              # (rl*rr) x r, orthonormal columns
            trans[t] = b1t.T.reshape(r, rl, rr)
    root = rng.standard_normal((1, rk(tr.left[0]), rk(tr.right[0])))

    # explicit nested bases of the root's two children
    def basis(t):
        if tr.is_leaf(t):
            return leaf[t]
        ul, ur = basis(tr.left[t]), basis(tr.right[t])
        b = trans[t]                                  # (r, rl, rr)
        kr = np.einsum("aj,bk->abjk", ul, ur).reshape(ul.shape[0] * ur.shape[0], -1)
        return kr @ b.reshape(b.shape[0], -1).T

    ul, ur = basis(tr.left[0]), basis(tr.right[0])
    dims = tuple([n] * order)
    N = n ** order
    scale = math.sqrt(N) / float(np.linalg.norm(root))
    X = np.empty(dims, dtype={"f64": np.float64, "f32": np.float32, "f16": np.float16,
                              "bf16": np.uint16}[dtype])
    nl = ul.shape[0]
    rows_per_slab = nl // n                               # slab = one index of mode 0
    mid = (root[0] * scale) @ ur.T                        # r_l x n_r

    def slab(i0):
        rows = ul[i0 * rows_per_slab:(i0 + 1) * rows_per_slab]
        t = rows @ mid
        if noise:
            t = t + noise * _rng(cfg, _NOISE, run, i0).standard_normal(t.shape)
        X[i0] = to_storage(t, dtype).reshape(dims[1:])

    _parallel_slabs(slab, n, threads)
    return HTInput(dims, X, dtype, tr, leaf, trans, root, scale, noise)


def inverse_norm_tensor(n: int, order: int, dtype: str = "f32", threads: int | None = None) -> np.ndarray:
    """X(i_1, .., i_d) = (i_1^2 + .. + i_d^2)^(-1/2) for i_j = 1..n: the function
    1 / ||x|| sampled on the uniform grid over [1, n]^d (the H-Tucker serial
    tests, Section 4.2.1).  Sums of squares are exact integers; each value is
    computed in FP64 and rounded once to the storage dtype."""
    if order < 2 or n < 1:
        raise ValueError("need order >= 2 and n >= 1")
    dims = (n,) * order
    X = np.empty(dims, dtype={"f64": np.float64, "f32": np.float32, "f16": np.float16,
                              "bf16": np.uint16}[dtype])
    sq = np.arange(1, n + 1, dtype=np.int64) ** 2
    rest = sq                                   # sums over modes 2..d, C-order
    for _ in range(order - 2):
        rest = (rest[:, None] + sq[None, :]).reshape(-1)

    def slab(i0):
        t = 1.0 / np.sqrt((sq[i0] + rest).astype(np.float64))
        X[i0] = to_storage(t, dtype).reshape(dims[1:])

    _parallel_slabs(slab, n, threads)
    return X


def node_sketches(dims, tree: DimTree, ells: dict, ws: dict, cfg: int, omega_dtype: str,
                  run: int = 0):
    """Sketch operands for every non-root node S: w_S sampled columns of X^(S)."""
    N = math.prod(dims)
    out = {}
    for t in range(1, tree.num_nodes):
        nS = math.prod(dims[k] for k in tree.modes(t))
        ncols = N // nS
        rng = _rng(cfg, _SKETCH, run, 1000 + t)
        w = min(int(ws[t]), ncols)
        idx = sample_columns(ncols, w, rng)
        out[t] = Sketch(idx, gaussian(w, int(ells[t]), rng, omega_dtype), omega_dtype)
    return out


# ---------------------------------------------------------------- batch specs
@dataclass
class BatchSpec:
    dims: tuple
    ranks: tuple
    ells: tuple
    ss: tuple


def batch_specs(count: int, cfg: int, nmin=16, nmax=96, rmin=4, rmax=16, p=5,
                cap=1 << 24, orders=(3, 4, 5)) -> list:
    """Uneven batch: order ~ U(orders), n_k ~ U[nmin, nmax] resampled until
    prod n_k <= cap, r_k ~ U[rmin, rmax] capped at n_k, ell_k = min(r_k+p, n_k),
    s_k = min(10 n_k, n_{!=k})."""
    rng = _rng(cfg, _BATCH)
    out = []
    for _ in range(count):
        d = int(rng.choice(orders))
        while True:
            dims = tuple(int(v) for v in rng.integers(nmin, nmax + 1, size=d))
            if math.prod(dims) <= cap:
                break
        ranks = tuple(min(int(v), n) for v, n in zip(rng.integers(rmin, rmax + 1, size=d), dims))
        ells = tuple(default_ell(dims, ranks, p))
        ss = tuple(max(e, s) for e, s in zip(ells, default_s(dims)))
        out.append(BatchSpec(dims, ranks, ells, ss))
    return out
