"""Seeded synthetic workloads shaped like the paper's experiments.

This module only *generates inputs*.  It holds none of the method's arithmetic
(no normalisation, no sketch, no distance, no profile): both the CPU oracle and
the HIP path receive the arrays it returns, so neither depends on the other.

Every workload is a multidimensional series T in R^{d x N} (Def. 1 of the
paper, Section II-B).  Several independent series can be concatenated along
time; ``offsets`` (length n_series+1) gives each series' column range, the
layout the C-ABI consumes.

Workload recipes (seeded numpy PCG64; data seed and sketch seed are recorded):

* ``random-walk-small``  random walk + sine per dimension, one planted chirp burst, d=8,
          n=4096, sum sketch k=1, m=64, excl=16 (Fig. 1 toy and Section IV-A
          random-walk generator).
* ``water-treatment``  water-treatment shaped (Section IV-D, SWaT has 51 sensors and
          actuators): 25 AR(1) sensors + 26 on/off actuators, d=51, n=50,000,
          three planted discords of length 100, Gaussian sketch k=8, m=100.
* ``transportation``  transportation shaped (Section IV-B, daily periodicity): d=1024,
          n=131,072, period 288, ten planted flattened/inverted days,
          Gaussian k=16, m=288.
* ``merchant-batch``  merchant shaped batch (Section I motivation, Section IV-C):
          4096 series, d=32, lengths U{2048..65536}, smoothed Poisson(3)
          counts in float32, spike bursts in 1% of series, Gaussian k=4, m=64.
* ``large-series``  large single series, random walk + sine, d=256, n=2^20, five planted
          discords of length 256, Gaussian k=32, m=256, plus an add/remove of
          16 dimensions (Section III-C).

``scale`` shrinks n (and the batch) so the same recipe yields small test cases.

``make_merchant_batch_device`` draws the full-size merchant batch (4.4e9 values) on a GPU
with torch's seeded generator instead of numpy (same recipe; the values differ
from ``make_merchant_batch``'s).  Checks that need the input on the host copy the series
they use back from the device tensor.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

__all__ = ["Workload", "make", "make_merchant_batch_device", "random_walk_sine", "tiny_series", "WORKLOADS"]


@dataclass
class Workload:
    name: str
    T: np.ndarray                 # d x N, float64 or float32, C-contiguous
    offsets: np.ndarray           # int64, n_series + 1
    dim_ids: np.ndarray           # int64, d (stable identifiers used by the hash)
    k: int
    kind: str                     # "sum" | "count" | "gauss"
    m: int
    excl: int
    sketch_seed: int
    data_seed: int
    precision: str                # path the recipe names: fp64 | fp32 | bf16x3 | fp16x3
    planted: List[Tuple[int, int, int, int]] = field(default_factory=list)  # (series, dim, offset, length)
    update: Optional[dict] = None  # large-series: {"T_add", "add_ids", "rem_ids"}

    @property
    def d(self) -> int:
        return int(self.T.shape[0])

    @property
    def n_series(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def cells(self) -> float:
        """k * n^2 / 2 summed over series (the throughput unit)."""
        L = self.lengths().astype(np.float64)
        return float(self.k * np.sum(L * L) / 2.0)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_walk_sine(rng: np.random.Generator, d: int, n: int, amp: float = 2.0) -> np.ndarray:
    """Gaussian random walk (step sigma 1) plus a sine of random period 50..400."""
    X = np.cumsum(rng.standard_normal((d, n)), axis=1)
    t = np.arange(n, dtype=np.float64)
    per = rng.uniform(50.0, 400.0, size=(d, 1))
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(d, 1))
    X += amp * np.sin(2.0 * np.pi * t[None, :] / per + ph)
    return X


def _nonoverlapping_offsets(rng, n: int, length: int, count: int, lo: int) -> List[int]:
    offs: List[int] = []
    tries = 0
    while len(offs) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("cannot place non-overlapping discords")
        o = int(rng.integers(lo, n - 2 * length))
        if all(abs(o - p) >= 2 * length for p in offs):
            offs.append(o)
    return offs


def _chirp_burst(x: np.ndarray, o: int, length: int, amp_sigmas: float) -> None:
    """Add a swept-frequency sine burst on [o, o+length) whose amplitude is
    amp_sigmas times the local sigma: the standard deviation of x over that
    window before insertion.

    The frequency sweeps from 1/32 upwards so that no shifted copy of the burst
    resembles it; a fixed-period burst whose period is below the trivial-match
    zone would be matched by its own shifted copies and would not be a discord.
    """
    s = float(np.std(x[o:o + length]))
    if s == 0.0:
        s = 1.0
    t = np.arange(length, dtype=np.float64)
    x[o:o + length] += amp_sigmas * s * np.sin(2.0 * np.pi * (t / 32.0 + t * t / (16.0 * length)))


def make_random_walk_small(scale: float = 1.0, data_seed: int = 1000, sketch_seed: int = 2000) -> Workload:
    rng = _rng(data_seed)
    d, m = 8, 64
    n = max(4 * m, int(4096 * scale))
    T = random_walk_sine(rng, d, n)
    o = int(rng.integers(m, n - 2 * m))
    _chirp_burst(T[0], o, m, 5.0)
    return Workload("random-walk-small", np.ascontiguousarray(T), np.array([0, n], np.int64), np.arange(d, dtype=np.int64),
                    k=1, kind="sum", m=m, excl=m // 4, sketch_seed=sketch_seed, data_seed=data_seed,
                    precision="fp64", planted=[(0, 0, o, m)])


def make_water_treatment(scale: float = 1.0, data_seed: int = 1001, sketch_seed: int = 2001) -> Workload:
    rng = _rng(data_seed)
    d_sens, d_act, m = 25, 26, 100
    n = max(8 * m, int(50_000 * scale))
    phi = 0.98
    X = np.empty((d_sens + d_act, n), np.float64)
    # AR(1) sensors with a stationary start, plus measurement noise
    e = rng.standard_normal((d_sens, n))
    x = rng.standard_normal(d_sens) / np.sqrt(1.0 - phi * phi)
    for t in range(n):  # vectorised over dims; n steps
        x = phi * x + e[:, t]
        X[:d_sens, t] = x
    X[:d_sens] += 0.1 * rng.standard_normal((d_sens, n))
    # on/off actuators: two-state Markov chain, switch probability 1/2000
    flips = rng.random((d_act, n)) < (1.0 / 2000.0)
    start = rng.integers(0, 2, size=(d_act, 1))
    X[d_sens:] = (start + np.cumsum(flips, axis=1)) % 2
    dims = rng.choice(d_sens + d_act, size=3, replace=False)
    offs = _nonoverlapping_offsets(rng, n, m, 3, m)
    planted = []
    for dim, o in zip(dims, offs):
        dim, o = int(dim), int(o)
        if dim < d_sens:
            _chirp_burst(X[dim], o, m, 5.0)
        else:
            t = np.arange(m)
            X[dim, o:o + m] = ((t // 10) % 2).astype(np.float64)  # square-wave chatter, period 20
        planted.append((0, dim, o, m))
    return Workload("water-treatment", np.ascontiguousarray(X), np.array([0, n], np.int64), np.arange(d_sens + d_act, dtype=np.int64),
                    k=8, kind="gauss", m=m, excl=m // 4, sketch_seed=sketch_seed, data_seed=data_seed,
                    precision="fp32", planted=planted)


def make_transportation(scale: float = 1.0, data_seed: int = 1002, sketch_seed: int = 2002) -> Workload:
    rng = _rng(data_seed)
    P, m = 288, 288
    d = max(8, int(1024 * min(1.0, scale * 4)))
    n = max(8 * m, int(131_072 * scale))
    u = np.arange(P, dtype=np.float64)
    f = np.sin(2 * np.pi * u / P) + 0.5 * np.sin(4 * np.pi * u / P + 1.0)  # two daily peaks
    amp = rng.lognormal(0.0, 0.5, size=(d, 1))
    ph = rng.integers(0, P, size=(d, 1))
    t = np.arange(n)
    X = amp * f[(t[None, :] + ph) % P] + 0.2 * rng.standard_normal((d, n))
    n_disc = 10 if n >= 40 * m else 2
    dims = rng.choice(d, size=n_disc, replace=False)
    offs = _nonoverlapping_offsets(rng, n, m, n_disc, m)
    planted = []
    for q, (dim, o) in enumerate(zip(dims, offs)):
        dim, o = int(dim), int(o)
        w = X[dim, o:o + m]
        mu = float(np.mean(w))
        if q % 2 == 0:
            X[dim, o:o + m] = mu + 0.2 * rng.standard_normal(m)   # flattened day
        else:
            X[dim, o:o + m] = 2.0 * mu - w                        # inverted day
        planted.append((0, dim, o, m))
    return Workload("transportation", np.ascontiguousarray(X), np.array([0, n], np.int64), np.arange(d, dtype=np.int64),
                    k=16, kind="gauss", m=m, excl=m // 4, sketch_seed=sketch_seed, data_seed=data_seed,
                    precision="bf16x3", planted=planted)


def make_merchant_batch(scale: float = 1.0, data_seed: int = 1003, sketch_seed: int = 2003,
            n_series: Optional[int] = None) -> Workload:
    rng = _rng(data_seed)
    d, m = 32, 64
    if n_series is None:
        n_series = max(4, int(4096 * scale))
    lo, hi = 2048, 65536
    if scale < 1.0:
        lo, hi = max(4 * m, int(lo * scale)), max(8 * m, int(hi * scale))
    L = rng.integers(lo, hi + 1, size=n_series)
    offsets = np.zeros(n_series + 1, np.int64)
    offsets[1:] = np.cumsum(L)
    N = int(offsets[-1])
    T = np.empty((d, N), np.float32)
    n_spiky = max(1, int(np.ceil(0.01 * n_series)))
    spiky = set(int(s) for s in rng.choice(n_series, size=n_spiky, replace=False))
    planted = []
    for s in range(n_series):
        a, b = int(offsets[s]), int(offsets[s + 1])
        Ls = b - a
        cnt = rng.poisson(3.0, size=(d, Ls)).astype(np.float64)
        if s in spiky:
            dim = int(rng.integers(0, d))
            o = int(rng.integers(0, Ls - m))
            pos = o + rng.choice(m, size=6, replace=False)
            cnt[dim, pos] += 20.0
            planted.append((s, dim, o, m))
        # 5-tap box filter with edge replication
        pad = np.concatenate([np.repeat(cnt[:, :1], 2, axis=1), cnt, np.repeat(cnt[:, -1:], 2, axis=1)], axis=1)
        cs = np.cumsum(pad, axis=1)
        cs = np.concatenate([np.zeros((d, 1)), cs], axis=1)
        T[:, a:b] = ((cs[:, 5:] - cs[:, :-5]) / 5.0).astype(np.float32)
    return Workload("merchant-batch", T, offsets, np.arange(d, dtype=np.int64), k=4, kind="gauss", m=m, excl=m // 4,
                    sketch_seed=sketch_seed, data_seed=data_seed, precision="fp32", planted=planted)


def make_large_series(scale: float = 1.0, data_seed: int = 1004, sketch_seed: int = 2004) -> Workload:
    rng = _rng(data_seed)
    d, m, n_upd = 256, 256, 16
    n = max(8 * m, int((1 << 20) * scale))
    T = random_walk_sine(rng, d, n)
    n_disc = 5
    dims = rng.choice(d, size=n_disc, replace=False)
    offs = _nonoverlapping_offsets(rng, n, m, n_disc, m)
    planted = []
    for dim, o in zip(dims, offs):
        _chirp_burst(T[int(dim)], int(o), m, 5.0)
        planted.append((0, int(dim), int(o), m))
    free = np.setdiff1d(np.arange(d), dims)
    rem_ids = np.sort(rng.choice(free, size=n_upd, replace=False)).astype(np.int64)
    T_add = random_walk_sine(_rng(data_seed + 500), n_upd, n)
    add_ids = np.arange(d, d + n_upd, dtype=np.int64)
    return Workload("large-series", np.ascontiguousarray(T), np.array([0, n], np.int64), np.arange(d, dtype=np.int64),
                    k=32, kind="gauss", m=m, excl=m // 4, sketch_seed=sketch_seed, data_seed=data_seed,
                    precision="fp16x3", planted=planted,
                    update={"T_add": np.ascontiguousarray(T_add), "add_ids": add_ids, "rem_ids": rem_ids})


def make_merchant_batch_device(torch, device, scale: float = 1.0, data_seed: int = 1003, sketch_seed: int = 2003,
                   n_series: Optional[int] = None):
    """The merchant-batch recipe drawn on ``device``: returns (Workload with T = None, T as a
    d x N float32 device tensor).  Lengths, spiky series and spike positions come
    from numpy (seeded); the Poisson counts from torch's generator seeded with
    data_seed; the 5-tap box filter replicates each series' edge samples."""
    rng = _rng(data_seed)
    d, m = 32, 64
    if n_series is None:
        n_series = max(4, int(4096 * scale))
    lo, hi = 2048, 65536
    if scale < 1.0:
        lo, hi = max(4 * m, int(lo * scale)), max(8 * m, int(hi * scale))
    L = rng.integers(lo, hi + 1, size=n_series)
    offsets = np.zeros(n_series + 1, np.int64)
    offsets[1:] = np.cumsum(L)
    N = int(offsets[-1])
    n_spiky = max(1, int(np.ceil(0.01 * n_series)))
    spiky = np.sort(rng.choice(n_series, size=n_spiky, replace=False))
    planted, rows, cols = [], [], []
    for s in spiky:
        dim = int(rng.integers(0, d))
        o = int(rng.integers(0, int(L[s]) - m))
        pos = o + rng.choice(m, size=6, replace=False)
        planted.append((int(s), dim, o, m))
        rows.extend([dim] * 6)
        cols.extend((offsets[s] + pos).tolist())
    g = torch.Generator(device=device)
    g.manual_seed(int(data_seed))
    cnt = torch.empty((d, N), dtype=torch.float32, device=device)
    for a in range(0, N, 1 << 26):  # chunks keep the rate tensor small
        b = min(N, a + (1 << 26))
        rate = torch.full((d, b - a), 3.0, dtype=torch.float32, device=device)
        cnt[:, a:b] = torch.poisson(rate, generator=g)
        del rate
    if rows:
        cnt[torch.tensor(rows, device=device), torch.tensor(cols, device=device)] += 20.0
    # 5-tap box filter over the concatenation, then the two samples at either
    # end of every series recomputed with that series' edge sample repeated
    T = torch.empty_like(cnt)
    T[:, 2:N - 2] = (cnt[:, 0:N - 4] + cnt[:, 1:N - 3] + cnt[:, 2:N - 2] + cnt[:, 3:N - 1] + cnt[:, 4:N]) / 5.0
    first = torch.from_numpy(offsets[:-1]).to(device)
    last = torch.from_numpy(offsets[1:] - 1).to(device)

    def col(ix):
        return cnt[:, ix]

    x0, x1, x2, x3 = col(first), col(first + 1), col(first + 2), col(first + 3)
    T[:, first] = (3 * x0 + x1 + x2) / 5.0
    T[:, first + 1] = (2 * x0 + x1 + x2 + x3) / 5.0
    y0, y1, y2, y3 = col(last), col(last - 1), col(last - 2), col(last - 3)
    T[:, last] = (3 * y0 + y1 + y2) / 5.0
    T[:, last - 1] = (2 * y0 + y1 + y2 + y3) / 5.0
    del cnt
    w = Workload("merchant-batch", None, offsets, np.arange(d, dtype=np.int64), k=4, kind="gauss", m=m, excl=m // 4,
                 sketch_seed=sketch_seed, data_seed=data_seed, precision="fp32", planted=planted)
    return w, T


WORKLOADS = {"random-walk-small": make_random_walk_small, "water-treatment": make_water_treatment, "transportation": make_transportation, "merchant-batch": make_merchant_batch, "large-series": make_large_series}


def make(name: str, scale: float = 1.0, **kw) -> Workload:
    return WORKLOADS[name](scale=scale, **kw)


def tiny_series(seed: int, d: int, n: int, kind: str = "rw") -> np.ndarray:
    """Small d x n test inputs: 'rw' random walk + sine, 'noise' iid N(0,1)."""
    rng = _rng(seed)
    if kind == "rw":
        return random_walk_sine(rng, d, n)
    if kind == "noise":
        return rng.standard_normal((d, n))
    raise ValueError(kind)
