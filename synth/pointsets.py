"""Batches of independent weighted point sets (robust-centre workload).

Each instance is a set of n points in R^d with positive weights: a unit
Gaussian cluster with a fraction of heavy-tailed outliers (multivariate
Student-t with nu degrees of freedom, scaled).  Layout matches the batched
solver's descriptors: all points concatenated point-major (instance b holds
n_b x d_b float32 values starting at ``a_off[b]``), weights concatenated at
``w_off[b]``, and a d_b-float slot for the result at ``z_off[b]``.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Mirrors em_instance_t of the C ABI: three int64 offsets then n and d (int32).
INSTANCE_DTYPE = np.dtype([("a_off", "<i8"), ("w_off", "<i8"), ("z_off", "<i8"),
                           ("n", "<i4"), ("d", "<i4")], align=True)
assert INSTANCE_DTYPE.itemsize == 32


@dataclass
class PointSetBatch:
    a: np.ndarray        # float32, concatenated points
    w: np.ndarray        # float32, concatenated weights
    inst: np.ndarray     # INSTANCE_DTYPE[B]
    z_size: int          # total floats of the z buffer (sum of d_b)
    lo: float
    hi: float

    @property
    def B(self) -> int:
        return int(self.inst.shape[0])

    def points(self, b: int) -> np.ndarray:
        e = self.inst[b]
        n, d = int(e["n"]), int(e["d"])
        return self.a[e["a_off"]:e["a_off"] + n * d].reshape(n, d)

    def weights(self, b: int) -> np.ndarray:
        e = self.inst[b]
        return self.w[e["w_off"]:e["w_off"] + int(e["n"])]

    def subset(self, idx) -> "PointSetBatch":
        """A compact batch holding only the instances ``idx`` (in that order)."""
        idx = np.asarray(idx, dtype=np.int64)
        pts = [self.points(int(b)) for b in idx]
        ws = [self.weights(int(b)) for b in idx]
        return pack_instances(pts, ws, self.lo, self.hi)


def pack_instances(points, weights, lo: float, hi: float) -> PointSetBatch:
    """Concatenate lists of (n_b x d_b) point arrays and n_b weight arrays."""
    B = len(points)
    inst = np.zeros(B, dtype=INSTANCE_DTYPE)
    a_sizes = np.array([p.size for p in points], dtype=np.int64)
    n = np.array([p.shape[0] for p in points], dtype=np.int64)
    d = np.array([p.shape[1] if p.ndim == 2 else 0 for p in points], dtype=np.int64)
    inst["a_off"] = np.concatenate([[0], np.cumsum(a_sizes)[:-1]]) if B else []
    inst["w_off"] = np.concatenate([[0], np.cumsum(n)[:-1]]) if B else []
    inst["z_off"] = np.concatenate([[0], np.cumsum(d)[:-1]]) if B else []
    inst["n"] = n
    inst["d"] = d
    a = np.concatenate([p.reshape(-1) for p in points]).astype(np.float32) if B else np.zeros(0, np.float32)
    w = np.concatenate([np.asarray(x).reshape(-1) for x in weights]).astype(np.float32) if B else np.zeros(0, np.float32)
    return PointSetBatch(a=a, w=w, inst=inst, z_size=int(d.sum()), lo=lo, hi=hi)


def _block(rng: np.random.Generator, B: int, n_lo: int, n_hi: int, d_choices,
           outlier_prob: float, nu: float, scale: float):
    n = rng.integers(n_lo, n_hi + 1, size=B)
    d = rng.choice(np.asarray(d_choices), size=B)
    pts, ws = [], []
    for b in range(B):
        nb, db = int(n[b]), int(d[b])
        Z = rng.standard_normal((nb, db))
        out = rng.uniform(size=nb) < outlier_prob
        V = rng.chisquare(nu, size=nb)
        mult = np.where(out, scale / np.sqrt(V / nu), 1.0)
        pts.append((Z * mult[:, None]).astype(np.float32))
        ws.append(rng.exponential(1.0, size=nb).astype(np.float32))
    return pts, ws


def make_pointset_batch(seed: int, B: int, n_lo: int = 8, n_hi: int = 512,
                        d_choices=(2, 3, 16, 49, 64), outlier_prob: float = 0.2,
                        nu: float = 1.5, scale: float = 50.0,
                        lo: float = -3.0, hi: float = 3.0,
                        block: int = 65536) -> PointSetBatch:
    """B instances: n ~ U{n_lo..n_hi}, d ~ U(d_choices), weights ~ Exp(1).

    Points: inliers ~ N(0, I_d); each point is an outlier with probability
    ``outlier_prob``, drawn as scale * Z / sqrt(V / nu) with Z ~ N(0, I_d) and
    V ~ chi^2_nu (one V per point: a multivariate Student-t).  Instances are
    drawn in blocks of ``block``, block j from SeedSequence(seed).spawn(...)[j],
    so every whole block is reproducible on its own.
    """
    nblk = max(1, -(-B // block))
    children = np.random.SeedSequence(seed).spawn(nblk)
    pts, ws = [], []
    left = B
    for j in range(nblk):
        m = min(block, left)
        left -= m
        p, w = _block(np.random.default_rng(children[j]), m, n_lo, n_hi, d_choices,
                      outlier_prob, nu, scale)
        pts += p
        ws += w
    return pack_instances(pts, ws, lo, hi)


def make_pointset_batch_device(seed: int, B: int, device, n_lo: int = 8, n_hi: int = 512,
                               d_choices=(2, 3, 16, 49, 64), outlier_prob: float = 0.2,
                               nu: float = 1.5, scale: float = 50.0):
    """The same distribution as make_pointset_batch, drawn on a torch device
    with a seeded torch generator (for full-size batches that do not fit a
    host-side draw in reasonable time).  Points of instances with equal d are
    stored contiguously (so per-point outlier scales broadcast), while the
    instance order is a random permutation.  Returns (a, w, inst_np,
    z_size): a and w are float32 device tensors, inst_np the descriptors
    (INSTANCE_DTYPE, host)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    n = torch.randint(n_lo, n_hi + 1, (B,), generator=g, device=device)
    dsel = torch.randint(0, len(d_choices), (B,), generator=g, device=device)
    dvals = torch.tensor(d_choices, device=device)[dsel]
    order = torch.randperm(B, generator=g, device=device)      # instance ids in storage order
    n_h = n.cpu().numpy().astype(np.int64)
    d_h = dvals.cpu().numpy().astype(np.int64)
    order_h = order.cpu().numpy()
    # storage: group by d (stable in the permuted order)
    grp = np.argsort(d_h[order_h], kind="stable")
    store = order_h[grp]                                        # instance ids, d-grouped
    sizes = n_h[store] * d_h[store]
    a_off_store = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    w_off_store = np.concatenate([[0], np.cumsum(n_h[store])[:-1]])
    inst = np.zeros(B, dtype=INSTANCE_DTYPE)
    inst["a_off"][store] = a_off_store
    inst["w_off"][store] = w_off_store
    inst["z_off"] = np.concatenate([[0], np.cumsum(d_h)[:-1]])
    inst["n"] = n_h
    inst["d"] = d_h
    total_a = int(sizes.sum())
    total_w = int(n_h.sum())
    a = torch.empty(total_a, dtype=torch.float32, device=device)
    w = torch.empty(total_w, dtype=torch.float32, device=device).exponential_(1.0, generator=g)
    pos_a = 0
    for dv in d_choices:
        sel = store[d_h[store] == dv]
        npts = int(n_h[sel].sum())
        if npts == 0:
            continue
        blk = a[pos_a:pos_a + npts * dv].view(npts, dv)
        blk.normal_(generator=g)
        out = torch.rand(npts, generator=g, device=device) < outlier_prob
        V = 2.0 * torch._standard_gamma(torch.full((npts,), nu / 2.0, device=device), generator=g)
        mult = torch.where(out, scale / torch.sqrt(V / nu), torch.ones_like(V))
        blk.mul_(mult[:, None])
        pos_a += npts * dv
    return a, w, inst, int(d_h.sum())
