"""Seeded synthetic workload generator (inputs only; none of the method's arithmetic).

Every column the tests and the benchmark use is a pure function of a seed and a
row index, so any single element can be recomputed on the host to check a
column that was generated on the device.

* Counter-based stream: ``x(seed, j) = splitmix64(seed + (j + 1) * 0x9E3779B97F4A7C15)``
  where splitmix64 is the finaliser published by Steele, Lea and Flood
  ("Fast splittable pseudorandom number generators", OOPSLA 2014).
* Uniform integer in ``[lo, hi]``: ``lo + (((x >> 32) * (hi - lo + 1)) >> 32)``
  (Lemire's multiply-shift on the top 32 bits; range at most 2**32).
* Zipf over ranks ``1..n`` with exponent ``s`` (Section 2.1: the frequency of
  rank r is proportional to r**-s): ``u = (x >> 11) * 2**-53`` and the sampled
  0-based rank is the smallest r with ``cdf[r] > u``, where ``cdf`` is the
  sequential float64 prefix sum of ``(r + 1)**-s`` divided by the total, with
  ``cdf[n-1] = 1.0``.  The table is built once, here, and uploaded as-is for
  the device sampler, so both sides compare the same doubles.
* Random permutation ``pi`` (rank -> key), standing in for the paper's "random
  order" of keys (Section 5.1): stable argsort of ``x(seed, j)``, j < n.
* Fact key ``j`` = ``pi[zipf_rank(j)]``.

The device half (``libskewgen.so``, built from ``csrc/workload_gen.hip``)
implements the same Zipf and uniform streams for columns too large to build on
the host; tests compare sampled device elements against this module.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seeds of the synthetic workloads (k = 1..5 for the five workload shapes).
def fact_seed(k: int) -> int:
    return 1000 + k


def perm_seed(k: int) -> int:
    return 2000 + k


def price_seed(k: int) -> int:
    return 3000 + k


def category_seed(k: int) -> int:
    return 3100 + k


def value_seed(k: int) -> int:
    return 4000 + k


def customer_seed(k: int) -> int:
    return 3200 + k


def splitmix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied elementwise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def stream(seed: int, start: int, n: int) -> np.ndarray:
    """x(seed, j) for j in [start, start + n)."""
    j = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return splitmix64(np.uint64(seed) + j * GOLDEN)


def uniform_int(seed: int, lo: int, hi: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform integers in [lo, hi] (inclusive), int64."""
    rng = hi - lo + 1
    if not (1 <= rng <= 2**32):
        raise ValueError("range must hold 1..2**32 values")
    x = stream(seed, start, n) >> np.uint64(32)
    with np.errstate(over="ignore"):
        off = (x * np.uint64(rng)) >> np.uint64(32)
    return off.astype(np.int64) + lo


def unit_double(x: np.ndarray) -> np.ndarray:
    return (x >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def zipf_cdf(n: int, s: float) -> np.ndarray:
    """Cumulative Zipf table over ranks 1..n (float64, last entry exactly 1.0)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)  # sequential accumulation, left to right
    cdf = c / c[-1]
    cdf[-1] = 1.0
    return cdf


def zipf_ranks(seed: int, cdf: np.ndarray, n: int, start: int = 0) -> np.ndarray:
    """0-based Zipf ranks for rows [start, start + n), int64."""
    u = unit_double(stream(seed, start, n))
    return np.searchsorted(cdf, u, side="right").astype(np.int64)


def permutation(seed: int, n: int) -> np.ndarray:
    """Seeded random permutation pi (rank -> key), int32."""
    return np.argsort(stream(seed, 0, n), kind="stable").astype(np.int32)


def fact_keys(seed: int, cdf: np.ndarray, pi: np.ndarray, n: int, start: int = 0) -> np.ndarray:
    """Zipf foreign keys: pi[rank] for rows [start, start + n), int32."""
    return pi[zipf_ranks(seed, cdf, n, start)].astype(np.int32)


def dimension(k: int, n_rows: int) -> tuple[np.ndarray, np.ndarray]:
    """Dimension columns of workload k: price U[1, 10000] int32, category U[0, 15] int8."""
    price = uniform_int(price_seed(k), 1, 10000, n_rows).astype(np.int32)
    cat = uniform_int(category_seed(k), 0, 15, n_rows).astype(np.int8)
    return price, cat


def harmonic(n: int, s: float) -> float:
    """Generalised harmonic number H_{n,s}."""
    return float(np.sum(np.arange(1, n + 1, dtype=np.float64) ** (-float(s))))


# ---------------------------------------------------------------------------
# Device half
# ---------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
GEN_LIB_PATH = os.path.join(_HERE, "lib", "libskewgen.so")
_gen_lib = None


def _device_lib():
    global _gen_lib
    if _gen_lib is None:
        import torch  # noqa: F401  (binds the HIP runtime torch already loaded)

        if not os.path.exists(GEN_LIB_PATH):
            raise RuntimeError(f"{GEN_LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(GEN_LIB_PATH)
        lib.skewgen_fact_keys.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_void_p]
        lib.skewgen_fact_keys.restype = ctypes.c_int
        lib.skewgen_uniform_i32.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_void_p]
        lib.skewgen_uniform_i32.restype = ctypes.c_int
        _gen_lib = lib
    return _gen_lib


def device_fact_keys(seed: int, cdf_dev, pi_dev, n: int, out=None, start: int = 0):
    """Generate fact keys on the current torch device (int32 tensor of length n)."""
    import torch

    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=cdf_dev.device)
    assert cdf_dev.dtype == torch.float64 and pi_dev.dtype == torch.int32
    assert cdf_dev.numel() == pi_dev.numel() and out.numel() >= n
    s = torch.cuda.current_stream(out.device).cuda_stream
    rc = _device_lib().skewgen_fact_keys(seed, cdf_dev.data_ptr(), cdf_dev.numel(), pi_dev.data_ptr(),
                                        out.data_ptr(), n, start, s)
    if rc != 0:
        raise RuntimeError(f"skewgen_fact_keys failed ({rc})")
    return out


def device_uniform_i32(seed: int, lo: int, hi: int, n: int, device, out=None, start: int = 0):
    import torch

    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=device)
    s = torch.cuda.current_stream(out.device).cuda_stream
    rc = _device_lib().skewgen_uniform_i32(seed, lo, hi, out.data_ptr(), n, start, s)
    if rc != 0:
        raise RuntimeError(f"skewgen_uniform_i32 failed ({rc})")
    return out


# ---------------------------------------------------------------------------
# Whole workloads (host or device resident)
# ---------------------------------------------------------------------------
def host_join_inputs(k: int, n_rows: int, n_fact: int, s: float):
    """Dimension (price, category) and Zipf fact keys of workload k, as numpy arrays."""
    cdf = zipf_cdf(n_rows, s)
    pi = permutation(perm_seed(k), n_rows)
    fact = fact_keys(fact_seed(k), cdf, pi, n_fact)
    price, cat = dimension(k, n_rows)
    return dict(fact=fact, price=price, category=cat, pi=pi, cdf=cdf)


def device_join_inputs(k: int, n_rows: int, n_fact: int, s: float, device="cuda"):
    """Same columns as host_join_inputs, with the fact column generated on the device."""
    import torch

    cdf = zipf_cdf(n_rows, s)
    pi = permutation(perm_seed(k), n_rows)
    price, cat = dimension(k, n_rows)
    cdf_d = torch.from_numpy(cdf).to(device)
    pi_d = torch.from_numpy(pi).to(device)
    fact = device_fact_keys(fact_seed(k), cdf_d, pi_d, n_fact)
    del cdf_d
    return dict(fact=fact, price=torch.from_numpy(price).to(device), category=torch.from_numpy(cat).to(device),
                pi=pi, cdf=cdf)


def host_group_inputs(k: int, n_groups: int, n_fact: int, s: float, vmax: int = 1000):
    cdf = zipf_cdf(n_groups, s)
    pi = permutation(perm_seed(k), n_groups)
    keys = fact_keys(fact_seed(k), cdf, pi, n_fact)
    vals = uniform_int(value_seed(k), 0, vmax, n_fact).astype(np.int32)
    return dict(keys=keys, vals=vals, pi=pi, cdf=cdf)


def device_group_inputs(k: int, n_groups: int, n_fact: int, s: float, vmax: int = 1000, device="cuda"):
    import torch

    cdf = zipf_cdf(n_groups, s)
    pi = permutation(perm_seed(k), n_groups)
    cdf_d = torch.from_numpy(cdf).to(device)
    pi_d = torch.from_numpy(pi).to(device)
    keys = device_fact_keys(fact_seed(k), cdf_d, pi_d, n_fact)
    del cdf_d
    vals = device_uniform_i32(value_seed(k), 0, vmax, n_fact, device)
    return dict(keys=keys, vals=vals, pi=pi, cdf=cdf)


# ---------------------------------------------------------------------------
# Batched star-join workload: a product dimension (price, category), a
# customer dimension (segment U[0, 99] int8), and a batch of fact tables of
# log-uniform sizes, each with a product key (Zipf s_prod through pi_p) and a
# customer key (Zipf s_cust through pi_c), stored one after the other.
# ---------------------------------------------------------------------------
def star_batch_spec(k: int, n_queries: int, fmin: float, fmax: float):
    """Row counts floor(fmin * (fmax / fmin) ** u) and customer thresholds U[1, 50] (1-50 % selectivity)."""
    u = unit_double(stream(5000 + k, 0, n_queries))
    sizes = np.floor(fmin * (fmax / fmin) ** u).astype(np.int64)
    lt = uniform_int(5100 + k, 1, 50, n_queries).astype(np.int32)
    start = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return sizes, lt, start


def star_dimensions(k: int, n_prod: int, n_cust: int):
    price, cat = dimension(k, n_prod)
    attr = uniform_int(customer_seed(k), 0, 99, n_cust).astype(np.int8)
    return price, cat, attr


def host_star_inputs(k: int, n_prod: int, n_cust: int, sizes, s_prod: float = 1.0, s_cust: float = 0.8):
    total = int(np.sum(sizes))
    pi_p = permutation(perm_seed(k), n_prod)
    pi_c = permutation(2100 + k, n_cust)
    prod = fact_keys(fact_seed(k), zipf_cdf(n_prod, s_prod), pi_p, total)
    cust = fact_keys(1100 + k, zipf_cdf(n_cust, s_cust), pi_c, total)
    price, cat, attr = star_dimensions(k, n_prod, n_cust)
    return dict(prod=prod, cust=cust, price=price, category=cat, cust_attr=attr)


def device_star_inputs(k: int, n_prod: int, n_cust: int, sizes, s_prod: float = 1.0, s_cust: float = 0.8,
                       device="cuda"):
    import torch

    total = int(np.sum(sizes))
    pi_p = torch.from_numpy(permutation(perm_seed(k), n_prod)).to(device)
    pi_c = torch.from_numpy(permutation(2100 + k, n_cust)).to(device)
    cdf = torch.from_numpy(zipf_cdf(n_prod, s_prod)).to(device)
    prod = device_fact_keys(fact_seed(k), cdf, pi_p, total)
    cdf = torch.from_numpy(zipf_cdf(n_cust, s_cust)).to(device)
    cust = device_fact_keys(1100 + k, cdf, pi_c, total)
    del cdf
    price, cat, attr = star_dimensions(k, n_prod, n_cust)
    return dict(prod=prod, cust=cust, price=torch.from_numpy(price).to(device),
                category=torch.from_numpy(cat).to(device), cust_attr=torch.from_numpy(attr).to(device))
