"""Planted LPs generated directly in device memory (torch's CUDA generator).

The same problem recipe as `lpgen.planted` (Gaussian A, planted optimum
(x*, y*, s*), b = A x*, c = A^T y* + s*), drawn with torch's counter-based CUDA
generator instead of numpy, so that the many large LPs of the batched and
serving workloads need no host generation or host-to-device copy.  These
problems are throughput stand-ins: they are not the numpy problems of the same
index, and parity tests use `lpgen.planted`.

Dense A is produced column-major ((n, m) row-major storage, FP32 values); b and
c are formed in FP64 from the FP32 values, a block of columns at a time.

Sparse A (the serving workload's CSR half) uses a stratified column pattern:
each of rows 0..m-2 gets k = round(density n) columns, one uniform column in
each of k equal strata of [0, n) (so the columns of a row are distinct and
sorted); the last row is all ones, as in `csr_planted`.
"""
from __future__ import annotations

import dataclasses


@dataclasses.dataclass
class DeviceLP:
    A: object            # dense: torch (m, n) view of column-major storage; CSR: (rowptr, colidx, vals)
    b: object            # torch float64 (m,)
    c: object            # torch float64 (n,)
    x_star: object
    y_star: object
    s_star: object
    m: int
    n: int
    w: int
    eps_gap: float
    seed: int
    a_dtype: str
    fmt: str
    opt: float
    name: str = ""

    @property
    def nbytes(self) -> int:
        if self.fmt == "dense":
            return self.A.numel() * self.A.element_size()
        return sum(t.numel() * t.element_size() for t in self.A)


def _plant_vectors(gen, m, n, support, torch, dev):
    supp = torch.randperm(n, generator=gen, device=dev)[:support]
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    x[supp] = torch.rand(support, generator=gen, device=dev, dtype=torch.float64)
    s = torch.rand(n, generator=gen, device=dev, dtype=torch.float64)
    s[supp] = 0.0
    y = torch.randn(m, generator=gen, device=dev, dtype=torch.float64)
    return x, y, s


def dense_planted_device(m, n, seed, support=None, w=None, eps_gap=1e-6, sketch_seed=0,
                         name="", dev="cuda") -> DeviceLP:
    import torch
    support = m if support is None else support
    block_cols = max(1024, (1 << 27) // m)   # FP64 staging of at most ~1 GiB
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    Acol = torch.randn((n, m), generator=gen, device=dev, dtype=torch.float32)
    x, y, s = _plant_vectors(gen, m, n, support, torch, dev)
    b = torch.zeros(m, dtype=torch.float64, device=dev)
    c = torch.empty(n, dtype=torch.float64, device=dev)
    for j0 in range(0, n, block_cols):
        blk = Acol[j0:j0 + block_cols].to(torch.float64)       # (cols, m)
        b += blk.t() @ x[j0:j0 + block_cols]
        c[j0:j0 + block_cols] = blk @ y + s[j0:j0 + block_cols]
        del blk
    opt = float(c @ x)
    return DeviceLP(Acol.t(), b, c, x, y, s, m, n, w if w else 4 * m, eps_gap, sketch_seed,
                    "f32", "dense", opt, name)


def csr_planted_device(m, n, density, seed, support=None, w=None, eps_gap=1e-6,
                       sketch_seed=0, name="", dev="cuda") -> DeviceLP:
    import torch
    support = m if support is None else support
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed))
    k = max(1, int(round(density * n)))
    # stratum edges floor(q n / k), q = 0..k: k non-empty strata when k <= n
    edges = (torch.arange(k + 1, device=dev, dtype=torch.int64) * n) // k
    lo, width = edges[:-1], edges[1:] - edges[:-1]
    u = torch.rand((m - 1, k), generator=gen, device=dev, dtype=torch.float64)
    cols = lo + torch.minimum((u * width).to(torch.int64), width - 1)
    vals = torch.randn((m - 1) * k, generator=gen, device=dev, dtype=torch.float32)
    colidx = torch.cat([cols.reshape(-1), torch.arange(n, device=dev, dtype=torch.int64)])
    vals = torch.cat([vals, torch.ones(n, device=dev, dtype=torch.float32)])
    rowptr = torch.empty(m + 1, dtype=torch.int64, device=dev)
    rowptr[:m] = torch.arange(m, device=dev, dtype=torch.int64) * k
    rowptr[m] = (m - 1) * k + n
    x, y, s = _plant_vectors(gen, m, n, support, torch, dev)
    rows = torch.repeat_interleave(torch.arange(m, device=dev),
                                   rowptr[1:] - rowptr[:-1])
    v64 = vals.to(torch.float64)
    b = torch.zeros(m, dtype=torch.float64, device=dev).index_add_(0, rows, v64 * x[colidx])
    c = torch.zeros(n, dtype=torch.float64, device=dev).index_add_(0, colidx, v64 * y[rows])
    c += s
    opt = float(c @ x)
    A = (rowptr.to(torch.int32), colidx.to(torch.int32), vals)
    return DeviceLP(A, b, c, x, y, s, m, n, w if w else 4 * m, eps_gap, sketch_seed, "f32",
                    "csr", opt, name)


def batch_lp_device(idx: int) -> DeviceLP:
    """LP `idx` of the batched workload (shapes from `lpgen.planted.batch_shape`)."""
    from .planted import batch_shape, sketch_seed
    m, k = batch_shape(idx)
    return dense_planted_device(m, m * k, seed=(3 << 32) + idx, w=4 * m, eps_gap=1e-6,
                                sketch_seed=sketch_seed(3, idx), name=f"batch{idx}")


def serving_lp_device(req: dict) -> DeviceLP:
    """Problem data of one serving request (see `lpgen.planted.serving_trace`)."""
    from .planted import sketch_seed
    idx, m, n = req["idx"], req["m"], req["n"]
    seed = (4 << 32) + idx
    if req["kind"] == "dense":
        return dense_planted_device(m, n, seed, w=4 * m, eps_gap=1e-6,
                                    sketch_seed=sketch_seed(4, idx), name=f"req{idx}")
    return csr_planted_device(m, n, 0.01, seed, w=4 * m, eps_gap=1e-6,
                              sketch_seed=sketch_seed(4, idx), name=f"req{idx}")
