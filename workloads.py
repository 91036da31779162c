"""Seeded synthetic workloads for the streaming IVF index.

This module only draws random inputs (vectors, ids, queries, centroids) with
the shapes and value distributions of the paper's workloads; it holds none of
the index's arithmetic.  Both the GPU library's tests/benchmark and the CPU
oracle are fed from here, so the two sides always see identical inputs.

Random streams: ``numpy.random.default_rng([seed, tag, ...])`` with
tag 0 = mixture means and base set, 1 = stream batch t, 2 = queries,
3 = operation choices, 4 = arrivals, 5 = k-means sample/initialisation.

Ids: the base set has ids 0..N-1 in generation order; stream batch t >= 1 adds
ids N + B*(t-1) + i, so "oldest" means the smallest live ids.

The paper's datasets (SIFT1M, Deep1B, ...) are not available; these mixtures
stand in for them (SIFT-like: d=128, integer values 0..255; Deep-like: d=96,
unit-normalised).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

L2, IP = 0, 1


@dataclass
class Workload:
    name: str
    dim: int
    nlist: int
    metric: int
    slab: int
    n_base: int
    batch: int
    n_queries: int
    nprobe: int
    k: int
    seed: int
    means: np.ndarray = field(repr=False)
    weights: np.ndarray = field(repr=False)
    sigma: float = 0.0
    kind: str = "gauss"          # gauss | gauss_int | vmf
    centroids: np.ndarray = field(default=None, repr=False)

    # -- sampling -------------------------------------------------------
    def _sample(self, rng, n):
        comp = rng.choice(self.means.shape[0], size=n, p=self.weights)
        if self.kind == "vmf":
            kappa = self.sigma
            x = self.means[comp].astype(np.float64) + rng.standard_normal((n, self.dim)) / np.sqrt(kappa)
            x /= np.linalg.norm(x, axis=1, keepdims=True)
            return x.astype(np.float32)
        x = self.means[comp].astype(np.float64) + self.sigma * rng.standard_normal((n, self.dim))
        if self.kind == "gauss_int":
            x = np.clip(np.rint(x), 0, 255)
        return x.astype(np.float32)

    def base(self, n=None, chunk=1 << 18):
        """Base set: (x[n, dim] float32, ids[n] int64)."""
        n = self.n_base if n is None else n
        rng = np.random.default_rng([self.seed, 0, 1])
        parts, left = [], n
        while left > 0:
            m = min(chunk, left)
            parts.append(self._sample(rng, m))
            left -= m
        x = np.concatenate(parts) if parts else np.zeros((0, self.dim), np.float32)
        return x, np.arange(n, dtype=np.int64)

    def stream_batch(self, t, b=None):
        """Batch t >= 1 of fresh vectors: (x[b, dim], ids[b])."""
        b = self.batch if b is None else b
        rng = np.random.default_rng([self.seed, 1, t])
        x = self._sample(rng, b)
        ids = self.n_base + self.batch * (t - 1) + np.arange(b, dtype=np.int64)
        return x, ids

    def oldest_ids(self, t, b=None):
        """Ids evicted at step t >= 1 (the oldest live batch)."""
        b = self.batch if b is None else b
        return b * (t - 1) + np.arange(b, dtype=np.int64)

    def queries(self, n=None, tag=0):
        n = self.n_queries if n is None else n
        rng = np.random.default_rng([self.seed, 2, tag])
        return self._sample(rng, n)


def _kmeans(sample, nlist, iters, seed):
    """Plain Lloyd iterations (numpy), used once to make fixed centroids.
    Init: nlist distinct sample rows; an empty cluster keeps its centroid.
    Nearest-centroid scoring uses float32 ||c||^2 - 2 x.c (the per-row ||x||^2
    does not change the argmin); means are accumulated in float64."""
    rng = np.random.default_rng([seed, 5])
    c = sample[rng.choice(sample.shape[0], size=nlist, replace=False)].astype(np.float64)
    xs32 = np.ascontiguousarray(sample, dtype=np.float32)
    xs = xs32.astype(np.float64)
    n, ch = xs32.shape[0], 8192
    a = np.empty(n, dtype=np.int64)
    sc = np.empty((ch, nlist), dtype=np.float32)
    for _ in range(iters):
        c32 = c.astype(np.float32)
        cc = (c32 * c32).sum(1)
        for s in range(0, n, ch):
            e = min(n, s + ch)
            np.matmul(xs32[s:e], c32.T, out=sc[:e - s])
            sc[:e - s] *= -2.0
            sc[:e - s] += cc[None, :]
            a[s:e] = sc[:e - s].argmin(1)
        sums = np.zeros_like(c)
        np.add.at(sums, a, xs)
        cnt = np.bincount(a, minlength=nlist)
        nz = cnt > 0
        c[nz] = sums[nz] / cnt[nz, None]
    return c.astype(np.float32)


def tiny(seed=0):
    """Tiny plain FP32: d=32, 16-component mixture, 4,096 base, slab 32."""
    rng = np.random.default_rng([seed, 0, 0])
    means = rng.uniform(-1.0, 1.0, size=(16, 32)).astype(np.float32)
    w = Workload("tiny", dim=32, nlist=16, metric=L2, slab=32, n_base=4096, batch=256,
                 n_queries=64, nprobe=4, k=10, seed=seed, means=means,
                 weights=np.full(16, 1.0 / 16), sigma=0.1, kind="gauss")
    w.centroids = means.copy()
    return w


def window(seed=0, n_base=1_000_000, kmeans_sample=65536, kmeans_iters=10):
    """Sliding window plain FP32: d=128 integer-valued 0..255, nlist 1,024
    (k-means, 10 iterations, seed 1), slab 64, +10k/-10k per step."""
    rng = np.random.default_rng([seed, 0, 0])
    means = rng.uniform(0.0, 255.0, size=(1024, 128)).astype(np.float32)
    w = Workload("window", dim=128, nlist=1024, metric=L2, slab=64, n_base=n_base, batch=10_000,
                 n_queries=10_000, nprobe=32, k=10, seed=seed, means=means,
                 weights=np.full(1024, 1.0 / 1024), sigma=48.0, kind="gauss_int")
    srng = np.random.default_rng([seed, 5, 0])
    sample = w._sample(srng, kmeans_sample)
    w.centroids = _kmeans(sample, 1024, kmeans_iters, seed=1)
    return w


def precision(seed=3, n_base=10_000_000):
    """Precision form inputs: d=96 unit vectors, 4,096-cluster vMF-like
    mixture (kappa 50), inner product, nlist 4,096, slab 128."""
    rng = np.random.default_rng([seed, 0, 0])
    mu = rng.standard_normal((4096, 96))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    w = Workload("precision", dim=96, nlist=4096, metric=IP, slab=128, n_base=n_base, batch=50_000,
                 n_queries=16_000, nprobe=64, k=10, seed=seed, means=mu.astype(np.float32),
                 weights=np.full(4096, 1.0 / 4096), sigma=50.0, kind="vmf")
    w.centroids = mu.astype(np.float32)
    return w


def batched(seed=4, n_base=5_000_000):
    """Batched uneven form inputs: d=128, Zipf(1.1) weights over 2,048
    clusters, nlist 2,048, slab 64; per-query nprobe and k vary."""
    rng = np.random.default_rng([seed, 0, 0])
    means = rng.uniform(0.0, 255.0, size=(2048, 128)).astype(np.float32)
    ranks = rng.permutation(2048)
    wts = (ranks + 1.0) ** -1.1
    wts /= wts.sum()
    w = Workload("batched", dim=128, nlist=2048, metric=L2, slab=64, n_base=n_base, batch=20_000,
                 n_queries=32_000, nprobe=128, k=100, seed=seed, means=means, weights=wts,
                 sigma=48.0, kind="gauss")
    w.centroids = means.copy()
    return w


def per_query_params(n, seed=4, nprobe_range=(8, 128), k_choices=(1, 10, 100)):
    """Per-query (nprobe, k) draws for the batched uneven form."""
    rng = np.random.default_rng([seed, 3, 0])
    npq = rng.integers(nprobe_range[0], nprobe_range[1] + 1, size=n).astype(np.int32)
    kpq = rng.choice(np.asarray(k_choices, dtype=np.int32), size=n).astype(np.int32)
    return npq, kpq


def random_live_ids(live_ids, n, seed, t):
    """n distinct ids drawn uniformly from the live id array (step t)."""
    rng = np.random.default_rng([seed, 3, t])
    return rng.choice(live_ids, size=n, replace=False).astype(np.int64)


def serving(seed=5, n_base=50_000_000):
    """Serving form inputs: d=128, 16,384 equal-weight clusters (means
    U[0,255]^128, sigma 48), L2, nlist 16,384 with the means as centroids,
    slab 128 (fp16 storage).  The base set and the payload pools are drawn on
    the device (``device_sample``): 50M host-side draws would take minutes."""
    rng = np.random.default_rng([seed, 0, 0])
    means = rng.uniform(0.0, 255.0, size=(16384, 128)).astype(np.float32)
    w = Workload("serving", dim=128, nlist=16384, metric=L2, slab=128, n_base=n_base, batch=0,
                 n_queries=4096, nprobe=64, k=10, seed=seed, means=means,
                 weights=np.full(16384, 1.0 / 16384), sigma=48.0, kind="gauss")
    w.centroids = means.copy()
    return w


def device_sample(w, n, tag, device, means=None):
    """n rows of the mixture drawn with torch's device generator (Philox),
    seeded by (w.seed, tag): float32 [n, dim] on ``device``.  Pass ``means``
    (the mixture means already on the device) to skip the copy."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(w.seed * 1_000_003 + tag)
    if means is None:
        means = torch.from_numpy(w.means).to(device)
    if np.allclose(w.weights, w.weights[0]):
        comp = torch.randint(0, w.means.shape[0], (n,), generator=g, device=device)
    else:   # skewed cluster weights (the batched form's Zipf mixture)
        wt = torch.from_numpy(w.weights).to(device=device, dtype=torch.float64)
        comp = torch.cat([torch.multinomial(wt, min(1 << 22, n - s), replacement=True, generator=g)
                          for s in range(0, n, 1 << 22)]) if n > 0 else torch.zeros(0, dtype=torch.int64,
                                                                                        device=device)
    x = torch.randn((n, w.dim), generator=g, device=device, dtype=torch.float32)
    x.mul_(w.sigma).add_(means[comp])
    return x


@dataclass
class Request:
    t: float            # arrival time (s) from the start of the stream
    kind: str           # "search" | "insert" | "delete"
    n: int              # queries, vectors or ids
    nprobe: int = 0
    oldest: bool = False


def serving_requests(duration_s, rate=2000.0, seed=5, mix=(0.5, 1 / 3, 1 / 6), insert_range=(1000, 50_000),
                     delete_range=(1000, 100_000), search_range=(1, 4096), nprobe_range=(16, 64)):
    """Poisson arrivals (exponential gaps, mean 1/rate) over duration_s with
    the serving mix: searches of log-uniform size with nprobe uniform,
    inserts and deletes of uniform size, deletes half oldest / half random."""
    rng = np.random.default_rng([seed, 4, 0])
    n_est = int(duration_s * rate * 1.2) + 64
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_est))
    t = t[t < duration_s]
    kinds = rng.choice(3, size=t.shape[0], p=np.asarray(mix) / np.sum(mix))
    lo, hi = np.log(search_range[0]), np.log(search_range[1] + 1)
    sq = np.minimum(np.floor(np.exp(rng.uniform(lo, hi, size=t.shape[0]))), search_range[1]).astype(int)
    sp = rng.integers(nprobe_range[0], nprobe_range[1] + 1, size=t.shape[0])
    si = rng.integers(insert_range[0], insert_range[1] + 1, size=t.shape[0])
    sd = rng.integers(delete_range[0], delete_range[1] + 1, size=t.shape[0])
    old = rng.random(t.shape[0]) < 0.5
    out = []
    for i in range(t.shape[0]):
        if kinds[i] == 0:
            out.append(Request(float(t[i]), "search", int(sq[i]), nprobe=int(sp[i])))
        elif kinds[i] == 1:
            out.append(Request(float(t[i]), "insert", int(si[i])))
        else:
            out.append(Request(float(t[i]), "delete", int(sd[i]), oldest=bool(old[i])))
    return out


def serving_delete_ids(reqs, n_base, seed=5):
    """Resolve every delete of a request stream to concrete ids, walking the
    stream in order (inserts take the next fresh ids).  Oldest deletes take
    the smallest live ids; random deletes draw ids uniformly from the live
    range (about as many as the request size are live) and keep the first
    r.n that are live at that point (a repeated draw stays in the request:
    removing an id twice is a no-op).  Returns {request index:
    int64 ids} and the number of ids live at the end."""
    rng = np.random.default_rng([seed, 3, 0])
    total = n_base + sum(r.n for r in reqs if r.kind == "insert")
    live = np.zeros(total, dtype=bool)
    live[:n_base] = True
    nxt, low, nlive = n_base, 0, n_base    # nlive: running estimate (repeated draws count twice)
    out = {}
    for i, r in enumerate(reqs):
        if r.kind == "insert":
            live[nxt:nxt + r.n] = True
            nxt += r.n
            nlive += r.n
        elif r.kind == "delete":
            if r.oldest:
                got, need = [], r.n
                while need > 0 and low < nxt:
                    seg = np.flatnonzero(live[low:min(nxt, low + max(2 * need, 4096))]) + low
                    take = seg[:need]
                    got.append(take)
                    need -= take.shape[0]
                    low = int(take[-1]) + 1 if take.shape[0] == seg.shape[0] and take.shape[0] else (
                        int(take[-1]) + 1 if take.shape[0] else min(nxt, low + max(2 * need, 4096)))
                ids = np.concatenate(got) if got else np.zeros(0, np.int64)
            else:
                # draw enough that about r.n of the draws are live
                frac = max(nlive, 1) / max(nxt - low, 1)
                cand = rng.integers(low, nxt, size=int(r.n / frac * 1.05) + 16) if nxt > low else \
                    np.zeros(0, np.int64)
                cand.sort()             # monotone addresses: far fewer cache and TLB misses
                ids = cand[live[cand]]
                if ids.shape[0] > r.n:
                    ids = ids[rng.permutation(ids.shape[0])[:r.n]]
                    ids.sort()
            live[ids] = False
            nlive -= ids.shape[0]
            out[i] = ids.astype(np.int64)
    return out, live
