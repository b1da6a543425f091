"""Seeded synthetic inputs for dominance aggregation.

Shared by the tests, the benchmark and the smoke check.  Holds no arithmetic of
the method: it only draws points and weights.  Every generator takes a seed and
uses numpy's PCG64, so the GPU path and the oracle see identical bytes.

Named workloads (the paper uses no dataset; these are synthetic stand-ins with
the sizes and distributions the build is measured on):

  int2d_64k        m=2, |D|=|Q|=65536, int32 coordinates U[0, 2^20) per axis
                   (ties present), int64 weights U[0, 1000)
  f32_2d_16m       m=2, |D|=|Q|=2^24, float32 coordinates U[0, 1) (a 2^-24 grid,
                   so ties occur), float32 weights N(0, 1)
  f32_3d_1m        m=3, |D|=|Q|=2^20, otherwise as f32_2d_16m
  f32_2d_4m_grad   m=2, |D|=|Q|=2^22, float32 U[0, 1), float32 weights N(0, 1)
                   and loss coefficients c ~ N(0, 1) per query
  batched_int2d    4096 instances, |D|=|Q|=round(2^U(8, 16)) per instance, int32
                   coordinates U[0, 2^16), int64 weights U[0, 1000)
  batched_gmm4d    64 instances, |D|=|Q|=round(2^U(12, 16)), m=4, float32 points
                   from a per-instance 8-component Gaussian mixture (means
                   U[0,1)^4, sigma 0.05, equal weights, shared by D and Q),
                   float32 weights N(0, 1) and int32 weights U[0, 1000)
"""
from __future__ import annotations

import dataclasses

import numpy as np

BASE_SEED = 16751


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Case:
    name: str
    m: int
    D: np.ndarray              # [nD, m]
    Q: np.ndarray              # [nQ, m]
    w: np.ndarray | None       # [nD]
    op: str = "sum"
    c: np.ndarray | None = None  # [nQ] loss coefficients (differentiable form)
    d_offsets: np.ndarray | None = None  # [n_inst + 1] (batched form)
    q_offsets: np.ndarray | None = None
    w_alt: np.ndarray | None = None      # second weight set (batched_gmm4d: int32)

    @property
    def n(self) -> int:
        return int(self.D.shape[0] + self.Q.shape[0])


def uniform_int_points(rng, n, m, hi, dtype=np.int32):
    return rng.integers(0, hi, size=(n, m), dtype=dtype)


def uniform_f32_points(rng, n, m):
    return rng.random((n, m), dtype=np.float32)


def int2d_64k(seed: int = BASE_SEED + 1, n: int = 65536) -> Case:
    rng = rng_for(seed)
    D = uniform_int_points(rng, n, 2, 1 << 20)
    Q = uniform_int_points(rng, n, 2, 1 << 20)
    w = rng.integers(0, 1000, size=n, dtype=np.int64)
    return Case("int2d_64k", 2, D, Q, w)


def f32_uniform(m: int, n: int, seed: int, name: str) -> Case:
    rng = rng_for(seed)
    D = uniform_f32_points(rng, n, m)
    Q = uniform_f32_points(rng, n, m)
    w = rng.standard_normal(n, dtype=np.float32)
    return Case(name, m, D, Q, w)


def f32_2d_16m(seed: int = BASE_SEED + 2, n: int = 1 << 24) -> Case:
    return f32_uniform(2, n, seed, "f32_2d_16m")


def f32_3d_1m(seed: int = BASE_SEED + 2, n: int = 1 << 20) -> Case:
    return f32_uniform(3, n, seed + 100, "f32_3d_1m")


def f32_2d_4m_grad(seed: int = BASE_SEED + 3, n: int = 1 << 22) -> Case:
    rng = rng_for(seed)
    D = uniform_f32_points(rng, n, 2)
    Q = uniform_f32_points(rng, n, 2)
    w = rng.standard_normal(n, dtype=np.float32)
    c = rng.standard_normal(n, dtype=np.float32)
    return Case("f32_2d_4m_grad", 2, D, Q, w, c=c)


def _log_uniform_sizes(rng, k, lo_exp, hi_exp):
    return np.rint(2.0 ** rng.uniform(lo_exp, hi_exp, size=k)).astype(np.int64)


def batched_int2d(seed: int = BASE_SEED + 4, n_inst: int = 4096,
                  lo_exp: float = 8, hi_exp: float = 16) -> Case:
    rng = rng_for(seed)
    s = _log_uniform_sizes(rng, n_inst, lo_exp, hi_exp)
    off = np.zeros(n_inst + 1, dtype=np.int64)
    off[1:] = np.cumsum(s)
    N = int(off[-1])
    D = uniform_int_points(rng, N, 2, 1 << 16)
    Q = uniform_int_points(rng, N, 2, 1 << 16)
    w = rng.integers(0, 1000, size=N, dtype=np.int64)
    return Case("batched_int2d", 2, D, Q, w, d_offsets=off, q_offsets=off.copy())


def _gmm_points(rng, n, means, sigma):
    comp = rng.integers(0, means.shape[0], size=n)
    x = means[comp] + sigma * rng.standard_normal((n, means.shape[1]))
    return x.astype(np.float32)


def batched_gmm4d(seed: int = BASE_SEED + 5, n_inst: int = 64,
                  lo_exp: float = 12, hi_exp: float = 16) -> Case:
    rng = rng_for(seed)
    s = _log_uniform_sizes(rng, n_inst, lo_exp, hi_exp)
    off = np.zeros(n_inst + 1, dtype=np.int64)
    off[1:] = np.cumsum(s)
    Ds, Qs = [], []
    for k in range(n_inst):
        means = rng.random((8, 4))
        Ds.append(_gmm_points(rng, int(s[k]), means, 0.05))
        Qs.append(_gmm_points(rng, int(s[k]), means, 0.05))
    D = np.concatenate(Ds)
    Q = np.concatenate(Qs)
    N = int(off[-1])
    w = rng.standard_normal(N, dtype=np.float32)
    w_alt = rng.integers(0, 1000, size=N, dtype=np.int32)
    return Case("batched_gmm4d", 4, D, Q, w, d_offsets=off, q_offsets=off.copy(),
                w_alt=w_alt)


def small_case(seed: int, m: int, nD: int, nQ: int, alphabet: int | None = 8,
               coord: str = "int", weight: str = "int64") -> Case:
    """Tiny inputs with heavy ties for oracle and parity checks.
    coord: 'int' (int32 values in [0, alphabet)) or 'f32' (float32 values on a
    grid of `alphabet` points in [0, 1), or U[0, 1) when alphabet is None).
    weight: 'int64', 'int32', 'f32', 'f64'."""
    rng = rng_for(seed)

    def pts(n):
        if coord == "int":
            return rng.integers(0, alphabet, size=(n, m), dtype=np.int32)
        if alphabet is None:
            return rng.random((n, m), dtype=np.float32)
        return (rng.integers(0, alphabet, size=(n, m)) / alphabet).astype(np.float32)

    D = pts(nD)
    Q = pts(nQ)
    if weight == "int64":
        w = rng.integers(-1000, 1000, size=nD, dtype=np.int64)
    elif weight == "int32":
        w = rng.integers(-1000, 1000, size=nD, dtype=np.int32)
    elif weight == "f32":
        w = rng.standard_normal(nD, dtype=np.float32)
    else:
        w = rng.standard_normal(nD)
    return Case(f"small_{m}d", m, D, Q, w)


def concat_instances(cases: list[Case]) -> tuple[np.ndarray, np.ndarray, np.ndarray,
                                                 np.ndarray, np.ndarray]:
    """Stack per-instance (D, Q, w) into the batched layout with offsets."""
    dof = np.zeros(len(cases) + 1, dtype=np.int64)
    qof = np.zeros(len(cases) + 1, dtype=np.int64)
    dof[1:] = np.cumsum([c.D.shape[0] for c in cases])
    qof[1:] = np.cumsum([c.Q.shape[0] for c in cases])
    D = np.concatenate([c.D for c in cases])
    Q = np.concatenate([c.Q for c in cases])
    w = np.concatenate([c.w for c in cases])
    return D, Q, w, dof, qof


WORKLOADS = {
    "int2d_64k": int2d_64k,
    "f32_2d_16m": f32_2d_16m,
    "f32_3d_1m": f32_3d_1m,
    "f32_2d_4m_grad": f32_2d_4m_grad,
    "batched_int2d": batched_int2d,
    "batched_gmm4d": batched_gmm4d,
}
