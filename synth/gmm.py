"""Seeded Gaussian-mixture vectors standing in for SIFT1B (u8, d=128), DEEP1B
(f32, d=96) and SPACEV1B (i8, d=100), the datasets of the paper's evaluation
(section 5.1), which are not available here.  Only their dtype, dimension and
query counts are copied; the value distributions are the mixture recipes below.

Recipes (component weights uniform; numpy PCG64):
  u8  : centres ~ U[40, 215]^d, x = rint(c + 20 z), clipped to [0, 255]
  i8  : centres ~ U[-88, 87]^d, x = rint(c + 20 z), clipped to [-128, 127]
  f32 : centres = normalize(N(0, I)), x = normalize(c + 0.1 z), in fp64, cast
  u8 with r latent dimensions (real descriptors vary along few directions
  within a cluster): per component a d x r basis B with N(0, 20^2 / r)
  entries, x = rint(c + B z_r + 2 z), clipped -- the same per-dimension spread
  as the u8 recipe, but of intrinsic dimension about r
Seeds: base 1000 + o, queries 2000 + o (graphs 3000 + o) for a workload with
seed offset o; the centres come from the base seed's first draws so that base
and queries share them.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    seed_offset: int
    name: str
    n: int
    d: int
    dtype: str          # "u8" | "i8" | "f32"
    components: int
    R: int
    slot: int           # record slot bytes
    tier: str           # "hbm" | "host" | "nvme"
    nq: int
    k: int
    L: tuple
    latent: int = 0     # u8 only: latent dimensions per component (0 = isotropic)

    @property
    def np_dtype(self):
        return {"u8": np.uint8, "i8": np.int8, "f32": np.float32}[self.dtype]


# The workloads of the measurements, named by what they are.
WORKLOADS = {
    "10k-u8-128": Workload(1, "10k u8/128, records in HBM", 10_000, 128, "u8", 16, 32, 256,
                           "hbm", 100, 10, (64,)),
    "1m-u8-128": Workload(2, "1M u8/128, records in pinned host DRAM", 1_000_000, 128, "u8",
                          256, 64, 512, "host", 10_000, 10, (32, 48, 64, 96, 128, 192, 256)),
    "10m-f32-96": Workload(3, "10M f32/96, 4 KB records in a file", 10_000_000, 96, "f32",
                           1024, 64, 4096, "nvme", 10_000, 10, (128,)),
    "100m-i8-100": Workload(4, "100M i8/100 batched, uneven L", 100_000_000, 100, "i8", 4096,
                            48, 512, "nvme", 100_000, 10, (32, 64, 128, 256)),
    "100m-u8-128": Workload(5, "100M u8/128 serving", 100_000_000, 128, "u8", 4096, 64, 512,
                            "nvme", 100_000, 10, (32, 64, 128, 256)),
    "1m-u8-128-latent16": Workload(6, "1M u8/128 of intrinsic dimension 16, records in pinned "
                                   "host DRAM", 1_000_000, 128, "u8", 256, 64, 512, "host",
                                   10_000, 10, (32, 48, 64, 96, 128, 192, 256), latent=16),
}


def _centres(rng: np.random.Generator, m: int, d: int, dtype: str) -> np.ndarray:
    if dtype == "u8":
        return rng.uniform(40.0, 215.0, size=(m, d))
    if dtype == "i8":
        return rng.uniform(-88.0, 87.0, size=(m, d))
    c = rng.standard_normal(size=(m, d))
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def _bases(rng: np.random.Generator, m: int, d: int, latent: int) -> np.ndarray:
    return rng.normal(0.0, 20.0 / np.sqrt(latent), size=(m, d, latent))


def _points(rng: np.random.Generator, centres: np.ndarray, n: int, dtype: str,
            chunk: int = 1 << 20, bases: np.ndarray | None = None) -> np.ndarray:
    m, d = centres.shape
    out = np.empty((n, d), dtype={"u8": np.uint8, "i8": np.int8, "f32": np.float32}[dtype])
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        comp = rng.integers(0, m, size=e - s)
        if dtype == "f32":
            x = centres[comp] + 0.1 * rng.standard_normal(size=(e - s, d))
            x /= np.linalg.norm(x, axis=1, keepdims=True)
            out[s:e] = x.astype(np.float32)
        elif bases is not None:
            r = bases.shape[2]
            z = rng.standard_normal(size=(e - s, r))
            x = centres[comp] + np.einsum("ndr,nr->nd", bases[comp], z)
            x = np.rint(x + 2.0 * rng.standard_normal(size=(e - s, d)))
            out[s:e] = np.clip(x, 0, 255).astype(out.dtype)
        else:
            x = np.rint(centres[comp] + 20.0 * rng.standard_normal(size=(e - s, d)))
            lo, hi = (0, 255) if dtype == "u8" else (-128, 127)
            out[s:e] = np.clip(x, lo, hi).astype(out.dtype)
    return out


def make_base(n: int, d: int, dtype: str, components: int, seed: int,
              latent: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = _centres(rng, components, d, dtype)
    bases = _bases(rng, components, d, latent) if latent else None
    return _points(rng, centres, n, dtype, bases=bases)


def make_queries(nq: int, d: int, dtype: str, components: int, base_seed: int,
                 query_seed: int, latent: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(base_seed))
    centres = _centres(rng, components, d, dtype)
    bases = _bases(rng, components, d, latent) if latent else None
    return _points(np.random.Generator(np.random.PCG64(query_seed)), centres, nq, dtype,
                   bases=bases)


def make_dataset(cfg: Workload, n: int | None = None, nq: int | None = None):
    """Base vectors and queries of workload ``cfg`` (optionally truncated sizes)."""
    n = cfg.n if n is None else n
    nq = cfg.nq if nq is None else nq
    base = make_base(n, cfg.d, cfg.dtype, cfg.components, 1000 + cfg.seed_offset, cfg.latent)
    queries = make_queries(nq, cfg.d, cfg.dtype, cfg.components, 1000 + cfg.seed_offset,
                           2000 + cfg.seed_offset, cfg.latent)
    return base, queries
