"""Seeded synthetic inputs (points + cluster labels) shared by the tests, the
benchmark and the CPU oracle's callers.

This module only draws data.  It contains none of the silhouette arithmetic
(no distances, no sampling probabilities, no estimators): the same arrays are
handed to the HIP path and to the FP64 oracle, which then compute
independently.

The paper evaluates on public UCI/SNAP datasets (n from hundreds to 6.4M,
z = 2..78, k = 2..20, Section 5.1.1, Table 2) clustered by k-means/k-medoids.
Those files are not available here; the generators below produce blob data of
the same shape family, with the recipes stated in each docstring.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "zipf_sizes", "gaussian_blobs", "vmf_blobs", "config_small", "config_zipf_gauss",
    "config_vmf_cos", "tiny_case",
]


def zipf_sizes(n: int, k: int, s: float = 1.1) -> np.ndarray:
    """Cluster sizes proportional to r^-s (r = 1..k), rounded with the
    largest-remainder rule so that they sum to exactly n (every size >= 1)."""
    w = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    raw = n * w / w.sum()
    base = np.floor(raw).astype(np.int64)
    rem = n - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    base = np.maximum(base, 1)
    # a size forced up to 1 is paid for by the largest cluster
    base[0] -= int(base.sum()) - n
    return base


def _shuffle(rng, X, labels):
    perm = rng.permutation(X.shape[0])
    return np.ascontiguousarray(X[perm]), np.ascontiguousarray(labels[perm])


def gaussian_blobs(n: int, d: int, k: int, seed: int, sizes=None, sigma=(1.0, 1.0),
                   center_range: float = 10.0, shuffle: bool = True):
    """Isotropic Gaussian blobs.

    centers ~ U[-center_range, center_range]^d; cluster j has standard
    deviation sigma_j ~ U[sigma[0], sigma[1]]; point = center + sigma_j*N(0, I).
    Returns (X float32 [n, d] row-major, labels int32 [n]); rows are shuffled by
    a seeded permutation so that clusters are interleaved in memory.
    """
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = np.full(k, n // k, dtype=np.int64)
        sizes[: n - int(sizes.sum())] += 1
    sizes = np.asarray(sizes, dtype=np.int64)
    assert int(sizes.sum()) == n and sizes.shape[0] == k
    centers = rng.uniform(-center_range, center_range, size=(k, d))
    sig = rng.uniform(sigma[0], sigma[1], size=k)
    X = np.empty((n, d), dtype=np.float32)
    labels = np.empty(n, dtype=np.int32)
    o = 0
    for j in range(k):
        m = int(sizes[j])
        X[o:o + m] = (centers[j] + sig[j] * rng.standard_normal((m, d))).astype(np.float32)
        labels[o:o + m] = j
        o += m
    if shuffle:
        X, labels = _shuffle(rng, X, labels)
    return X, labels


def _wood_vmf(rng, mu: np.ndarray, kappa: float, m: int) -> np.ndarray:
    """m draws from the von Mises-Fisher distribution on S^{d-1} with mean
    direction mu and concentration kappa (Wood, 1994, rejection sampler for
    the component along mu, uniform direction in the orthogonal complement)."""
    d = mu.shape[0]
    dm1 = d - 1.0
    b = (-2.0 * kappa + np.sqrt(4.0 * kappa * kappa + dm1 * dm1)) / dm1
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + dm1 * np.log(1.0 - x0 * x0)
    w = np.empty(m)
    got = 0
    while got < m:
        need = m - got
        batch = int(need * 1.3) + 16
        z = rng.beta(dm1 / 2.0, dm1 / 2.0, size=batch)
        ww = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        u = rng.uniform(size=batch)
        ok = kappa * ww + dm1 * np.log(1.0 - x0 * ww) - c >= np.log(u)
        acc = ww[ok][:need]
        w[got:got + acc.shape[0]] = acc
        got += acc.shape[0]
    v = rng.standard_normal((m, d))
    v -= np.outer(v @ mu, mu)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return w[:, None] * mu[None, :] + np.sqrt(np.maximum(0.0, 1.0 - w * w))[:, None] * v


def vmf_blobs(n: int, d: int, k: int, seed: int, kappa: float = 50.0, sizes=None,
              shuffle: bool = True):
    """Directional blobs: mean directions uniform on S^{d-1}; cluster j draws
    from vMF(mu_j, kappa) (Wood's sampler); rows are L2-normalised in float64
    before the cast to float32."""
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = zipf_sizes(n, k)
    sizes = np.asarray(sizes, dtype=np.int64)
    X = np.empty((n, d), dtype=np.float32)
    labels = np.empty(n, dtype=np.int32)
    o = 0
    for j in range(k):
        mu = rng.standard_normal(d)
        mu /= np.linalg.norm(mu)
        m = int(sizes[j])
        P = _wood_vmf(rng, mu, kappa, m)
        P /= np.linalg.norm(P, axis=1, keepdims=True)
        X[o:o + m] = P.astype(np.float32)
        labels[o:o + m] = j
        o += m
    if shuffle:
        X, labels = _shuffle(rng, X, labels)
    return X, labels


def config_small():
    """n=2,000, d=8, k=4 equal Gaussian blobs (sigma=1, centers U[-10,10]^8), seed 0."""
    return gaussian_blobs(2000, 8, 4, seed=0)


def config_zipf_gauss(n: int = 1_000_000, d: int = 32, k: int = 16, seed: int = 1):
    """n=1e6, d=32, k=16 Gaussian blobs, Zipf(1.1) sizes, sigma_j ~ U[0.5, 2], seed 1."""
    return gaussian_blobs(n, d, k, seed=seed, sizes=zipf_sizes(n, k), sigma=(0.5, 2.0))


def config_vmf_cos(n: int = 4_000_000, d: int = 128, k: int = 64, seed: int = 2):
    """n=4e6, d=128, k=64 vMF(kappa=50) blobs with Zipf(1.1) sizes, unit rows, seed 2."""
    return vmf_blobs(n, d, k, seed=seed, kappa=50.0, sizes=zipf_sizes(n, k))


def tiny_case(n: int, d: int, k: int, seed: int, sigma=(0.5, 2.0), sizes=None):
    """Small Gaussian-blob case for parity tests (uneven sizes by default)."""
    if sizes is None:
        rng = np.random.default_rng(seed + 7919)
        w = rng.uniform(0.3, 1.0, size=k)
        sizes = np.maximum(1, np.floor(n * w / w.sum()).astype(np.int64))
        sizes[0] += n - int(sizes.sum())
    return gaussian_blobs(n, d, k, seed=seed, sizes=sizes, sigma=sigma)


def split_blobs(n: int, d: int, k: int, seed: int, sep: float = 100.0, tight: float = 0.01,
                offset: float = 1000.0, dup: float = 0.0):
    """Cluster 0 is two tight blobs (sigma = `tight`) `sep` apart, so its
    centre lies far from every one of its points while their near neighbours
    are close; clusters 1..k-1 are ordinary blobs (sigma 1) around centres
    U[-sep, sep]^d.  Everything is shifted by `offset` in every coordinate.
    With dup > 0 every second row of cluster 0 is a copy of the row before it
    moved by N(0, dup^2) per coordinate (near-duplicate pairs).  Rows are
    shuffled; half the rows belong to cluster 0."""
    rng = np.random.default_rng(seed)
    n0 = n // 2
    rest = n - n0
    sizes = np.full(k - 1, rest // (k - 1))
    sizes[0] += rest - int(sizes.sum())
    c0 = rng.uniform(-sep, sep, size=d)
    direc = rng.standard_normal(d)
    direc /= np.linalg.norm(direc)
    half = n0 // 2
    A = c0 + rng.normal(scale=tight, size=(half, d))
    B = c0 + sep * direc + rng.normal(scale=tight, size=(n0 - half, d))
    X0 = np.concatenate([A, B])
    if dup > 0.0:
        X0[1::2] = X0[0:-1:2][: X0[1::2].shape[0]] + rng.normal(scale=dup, size=X0[1::2].shape)
    parts = [X0]
    labels = [np.zeros(n0, dtype=np.int32)]
    for j in range(1, k):
        cj = rng.uniform(-sep, sep, size=d)
        parts.append(cj + rng.normal(size=(int(sizes[j - 1]), d)))
        labels.append(np.full(int(sizes[j - 1]), j, dtype=np.int32))
    X = (np.concatenate(parts) + offset).astype(np.float32)
    L = np.concatenate(labels)
    return _shuffle(rng, X, L)


# ---------------------------------------------------------------------------
# Exponential blobs and Voronoi clusterings (the k-sweep workload), and the
# serving workload's dataset pool and request stream.
# ---------------------------------------------------------------------------
def exp_blobs(n: int, d: int, blobs: int, seed: int, offset_range=(0.0, 10.0)):
    """x = o_b + Exp(1) per coordinate, o_b ~ U[offset_range]^d, each row in
    one of `blobs` blobs chosen uniformly (positive data, for Canberra)."""
    rng = np.random.default_rng(seed)
    offs = rng.uniform(offset_range[0], offset_range[1], size=(blobs, d))
    which = rng.integers(0, blobs, size=n)
    X = offs[which] + rng.exponential(1.0, size=(n, d))
    return np.ascontiguousarray(X.astype(np.float32))


def voronoi_centers(n: int, k: int, seed) -> np.ndarray:
    """k distinct row indices drawn with the given seed (an int or a tuple)."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=k, replace=False))


def voronoi_labels(X, centers, chunk: int = 1 << 16):
    """Nearest center by Euclidean distance (ties to the lowest index), on the
    host in float64; X [n][d], centers: row indices."""
    X = np.asarray(X, dtype=np.float64)
    C = X[np.asarray(centers)]
    cn = (C * C).sum(axis=1)
    out = np.empty(X.shape[0], dtype=np.int32)
    for r0 in range(0, X.shape[0], chunk):
        xb = X[r0:r0 + chunk]
        d2 = (xb * xb).sum(axis=1)[:, None] - 2.0 * xb @ C.T + cn[None, :]
        out[r0:r0 + chunk] = np.argmin(d2, axis=1)
    return out


def voronoi_labels_device(X, centers, chunk: int = 1 << 18):
    """The same clustering rule on a device tensor X (float32 arithmetic;
    used for large inputs that are only checked against themselves)."""
    import torch
    C = X[torch.as_tensor(np.asarray(centers), device=X.device, dtype=torch.long)]
    cn = (C * C).sum(dim=1)
    out = torch.empty(X.shape[0], dtype=torch.int32, device=X.device)
    for r0 in range(0, X.shape[0], chunk):
        xb = X[r0:r0 + chunk]
        d2 = (xb * xb).sum(dim=1, keepdim=True) - 2.0 * (xb @ C.T) + cn[None, :]
        out[r0:r0 + chunk] = torch.argmin(d2, dim=1).to(torch.int32)
    return out


def config_sweep(n: int = 500_000, d: int = 64, blobs: int = 16, seed: int = 3):
    """k-sweep data: exponential blobs (their Voronoi clusterings for
    k = 2..257 come from voronoi_centers(n, k, (seed, k)))."""
    return exp_blobs(n, d, blobs, seed)


SERVING_METRICS = ("eucl", "cos", "manh", "canb")


def serving_pool_specs(count: int = 32, seed: int = 5, dims=(16, 64, 256), n_range=(1e4, 2e6)):
    """The resident datasets of the serving workload: n = round(10^U[log10
    n_range]), d from dims, a metric each (its data family follows it)."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = int(round(10.0 ** rng.uniform(np.log10(n_range[0]), np.log10(n_range[1]))))
        specs.append({"id": i, "n": n, "d": int(rng.choice(dims)),
                      "metric": SERVING_METRICS[int(rng.integers(0, 4))], "seed": 100 + i})
    return specs


def serving_dataset(spec, device):
    """Generate one serving dataset on the device (torch generator, seeded):
    Zipf Gaussian blobs (Euclidean / Manhattan; rows scaled to unit length for
    cosine) or exponential blobs (Canberra)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(spec["seed"]))
    n, d = spec["n"], spec["d"]
    if spec["metric"] == "canb":
        offs = torch.rand((16, d), generator=g, device=device) * 10.0
        which = torch.randint(0, 16, (n,), generator=g, device=device)
        X = offs[which] + torch.empty((n, d), device=device).exponential_(1.0, generator=g)
        return X.contiguous()
    k = 16
    sizes = torch.as_tensor(zipf_sizes(n, k), device=device)
    centers = torch.rand((k, d), generator=g, device=device) * 20.0 - 10.0
    sig = torch.rand((k,), generator=g, device=device) * 1.5 + 0.5
    lab = torch.repeat_interleave(torch.arange(k, device=device), sizes)
    X = centers[lab] + sig[lab, None] * torch.randn((n, d), generator=g, device=device)
    X = X[torch.randperm(n, generator=g, device=device)]
    if spec["metric"] == "cos":
        X = X / X.norm(dim=1, keepdim=True).clamp_min(1e-30)
    return X.contiguous()


def serving_requests(specs, count: int, seed: int = 7, ks=(2, 128), ts=(64, 256, 1024)):
    """Request stream: dataset uniform, k ~ U{ks}, t from ts, Philox seed
    1000 + request id; the clustering is the Voronoi partition of k rows
    drawn with seed (request seed, k)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(count):
        spec = specs[int(rng.integers(0, len(specs)))]
        k = int(rng.integers(ks[0], ks[1] + 1))
        reqs.append({"id": i, "dataset": spec["id"], "k": k, "t": int(rng.choice(ts)), "seed": 1000 + i,
                     "centers_seed": (1000 + i, k)})
    return reqs
