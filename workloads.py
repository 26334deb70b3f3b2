"""Seeded synthetic particle sets for the octree build.

This module is shared by the tests, the benchmark, the oracle checks and the
GPU path as the single source of input data. It holds none of the method's
arithmetic (no keys, sorting or trees): it only draws particle coordinates.

Every host generator is deterministic in (seed, stream): numpy's Philox
(4x64, 10 rounds) counter-based bit generator keyed by the seed, with the
stream number as the counter's starting block, so any set can be regenerated
on its own. The device generator (workloads_gpu.hip, for workloads too large
to draw on the host) uses Philox4x32-10 keyed by (seed, stream) with the same
recipes; its sets are copied back to the host whenever an oracle checks them.

Recipes (shapes of the workloads the octree build is measured on):
  * uniform cube: x, y, z i.i.d. uniform in [0, 1), each drawn as
    (u64 >> 11) * 2^-53 so every value is an exact double;
  * Plummer sphere (scale radius a, truncated at r_t): radius by inverting the
    cumulative mass M(r) = r^3 / (a^2 + r^2)^(3/2) on X ~ U(0, M(r_t)), then an
    isotropic direction (cos(theta) = 2u - 1, phi = 2 pi v);
  * Gaussian displacement: every coordinate moved by N(0, sigma^2).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
GPU_SRC = os.path.join(_HERE, "workloads_gpu.hip")
GPU_LIB = os.path.join(_HERE, "libworkloads_gpu.so")
KINDS = {"uniform": 0, "plummer": 1}

UNIT_BOX = ((0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
PLUMMER_RT = 20.0
PLUMMER_BOX = ((-PLUMMER_RT,) * 3, (PLUMMER_RT,) * 3)

_STREAM_STRIDE = 1 << 40  # Philox blocks reserved per stream


def _gen(seed: int, stream: int = 0) -> np.random.Generator:
    bg = np.random.Philox(key=int(seed))
    if stream:
        bg = bg.advance(int(stream) * _STREAM_STRIDE)
    return np.random.Generator(bg)


def _unit_doubles(g: np.random.Generator, n: int) -> np.ndarray:
    raw = g.bit_generator.random_raw(n)
    return (raw >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_cube(n: int, seed: int, stream: int = 0):
    """n particles i.i.d. uniform in [0, 1)^3 (x, y, z float64 arrays)."""
    g = _gen(seed, stream)
    u = _unit_doubles(g, 3 * n)
    return u[0::3].copy(), u[1::3].copy(), u[2::3].copy()


def plummer_sphere(n: int, seed: int, stream: int = 0, a: float = 1.0, r_t: float = PLUMMER_RT):
    """n particles from a Plummer sphere of scale radius a truncated at r_t."""
    g = _gen(seed, stream)
    u = _unit_doubles(g, 3 * n)
    x_max = r_t ** 3 / (a * a + r_t * r_t) ** 1.5
    X = (u[0::3] * x_max).clip(1e-300, None)
    r = a / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    cos_t = 2.0 * u[1::3] - 1.0
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    phi = 2.0 * math.pi * u[2::3]
    return r * sin_t * np.cos(phi), r * sin_t * np.sin(phi), r * cos_t


def gaussian_displace(x, y, z, sigma: float, seed: int, stream: int):
    """Copy of (x, y, z) with every coordinate moved by N(0, sigma^2)."""
    g = _gen(seed, stream)
    d = g.standard_normal(3 * x.size) * sigma
    return x + d[0::3], y + d[1::3], z + d[2::3]


@dataclass(frozen=True)
class ParticleSet:
    """One tree-build instance: particles, bounding box, curve, N_crit."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    box: tuple
    curve: int  # 0 Morton, 1 Hilbert
    n_crit: int
    kind: str

    @property
    def n(self) -> int:
        return int(self.x.size)


MORTON, HILBERT = 0, 1


def make_set(kind: str, n: int, seed: int, stream: int, curve: int, n_crit: int) -> ParticleSet:
    if kind == "uniform":
        x, y, z = uniform_cube(n, seed, stream)
        box = UNIT_BOX
    elif kind == "plummer":
        x, y, z = plummer_sphere(n, seed, stream)
        box = PLUMMER_BOX
    else:
        raise ValueError(kind)
    return ParticleSet(x, y, z, box, curve, n_crit, kind)


# ---- The measured configurations ------------------------------------------

def config_small(seed: int = 1) -> ParticleSet:
    """65,536 uniform particles, Morton keys, N_crit = 64."""
    return make_set("uniform", 1 << 16, seed, 0, MORTON, 64)


def config_uniform_2_24(seed: int = 2, n: int = 1 << 24) -> ParticleSet:
    """2^24 uniform particles, Hilbert keys, N_crit = 64 (the benchmarked build)."""
    return make_set("uniform", n, seed, 0, HILBERT, 64)


def config_plummer(seed: int = 3, n: int = 1 << 27) -> ParticleSet:
    """2^27 Plummer particles (a = 1, r_t = 20), Hilbert keys, N_crit = 16."""
    return make_set("plummer", n, seed, 0, HILBERT, 16)


def plummer_rebuild_steps(s: ParticleSet, steps: int = 10, sigma: float = 1e-3, seed: int = 3):
    """Cumulative Gaussian displacements of a Plummer set, one per rebuild."""
    x, y, z = s.x, s.y, s.z
    for k in range(1, steps + 1):
        x, y, z = gaussian_displace(x, y, z, sigma, seed, k)
        yield ParticleSet(x, y, z, s.box, s.curve, s.n_crit, s.kind)


def batched_specs(count: int = 512, seed: int = 4, log2_min: float = 10.0, log2_max: float = 20.0):
    """Per-instance (kind, n, curve, n_crit, stream) for the batched workload:
    sizes floor(2^U), U ~ U[log2_min, log2_max]; uniform or Plummer and Morton or
    Hilbert by coin flip; N_crit from {8, 16, 32, 64, 128}."""
    g = _gen(seed, 0)
    U = g.uniform(log2_min, log2_max, count)
    kinds = g.integers(0, 2, count)
    curves = g.integers(0, 2, count)
    ncrits = np.array([8, 16, 32, 64, 128])[g.integers(0, 5, count)]
    return [("plummer" if kinds[s] else "uniform", int(2.0 ** U[s]), int(curves[s]), int(ncrits[s]), s + 1)
            for s in range(count)]


def batched_sets(count: int = 512, seed: int = 4, **kw):
    return [make_set(kind, n, seed, stream, curve, nc) for kind, n, curve, nc, stream in
            batched_specs(count, seed, **kw)]


def serving_specs(count: int = 10000, seed: int = 5, log2_min: float = 12.0, log2_max: float = 22.0):
    """Per-request (kind, n, n_crit, stream, interarrival_unit) for the serving
    workload: sizes floor(2^U), U ~ U[log2_min, log2_max]; uniform or Plummer;
    Hilbert keys; N_crit in {16, 64}; unit-mean exponential inter-arrival gaps
    (scaled by the caller to the chosen arrival rate)."""
    g = _gen(seed, 0)
    U = g.uniform(log2_min, log2_max, count)
    kinds = g.integers(0, 2, count)
    ncrits = np.array([16, 64])[g.integers(0, 2, count)]
    gaps = g.exponential(1.0, count)
    return [("plummer" if kinds[s] else "uniform", int(2.0 ** U[s]), int(ncrits[s]), s + 1, float(gaps[s]))
            for s in range(count)]


# ---- device generator --------------------------------------------------------------

def build_gpu_generator() -> str:
    """Compile workloads_gpu.hip for gfx950 into libworkloads_gpu.so."""
    cmd = ["hipcc", "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-fvisibility=hidden",
           GPU_SRC, "-o", GPU_LIB]
    subprocess.run(cmd, check=True)
    return GPU_LIB


_gpu = None


def _gpu_lib():
    global _gpu
    if _gpu is None:
        if not os.path.exists(GPU_LIB):
            raise ImportError(f"{GPU_LIB} is missing: run workloads.build_gpu_generator()")
        lib = ctypes.CDLL(GPU_LIB)
        P = ctypes.c_void_p
        lib.wl_generate.restype = ctypes.c_int
        lib.wl_generate.argtypes = [P, P, P, P, P, ctypes.c_uint32, P, P, P, P]
        lib.wl_displace.restype = ctypes.c_int
        lib.wl_displace.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32, P]
        lib.wl_philox.restype = ctypes.c_int
        lib.wl_philox.argtypes = [P, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, P, P]
        _gpu = lib
    return _gpu


def device_generate(sets, x, y, z, stream=None, base: int = 0):
    """Draw sets [(kind, n, seed, stream), ...] back to back into the float64
    device tensors x, y, z starting at element `base`; returns the offsets
    (n_sets + 1, relative to base). Asynchronous on `stream`."""
    import torch

    k = len(sets)
    counts = np.array([int(s[1]) for s in sets], dtype=np.uint64)
    offs = np.zeros(k + 1, dtype=np.uint64)
    np.cumsum(counts, out=offs[1:])
    assert x.numel() >= base + int(offs[-1]) and x.dtype == torch.float64
    kinds = np.array([KINDS[s[0]] for s in sets], dtype=np.uint32)
    seeds = np.array([int(s[2]) for s in sets], dtype=np.uint32)
    streams = np.array([int(s[3]) for s in sets], dtype=np.uint32)
    o = offs[:-1] + np.uint64(base)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = _gpu_lib().wl_generate(o.ctypes.data, counts.ctypes.data, kinds.ctypes.data, seeds.ctypes.data,
                                streams.ctypes.data, k, x.data_ptr(), y.data_ptr(), z.data_ptr(), st.cuda_stream)
    if rc != 0:
        raise RuntimeError("wl_generate failed")
    return offs.astype(np.int64)


def device_sets(sets, device="cuda"):
    """Allocate and draw sets [(kind, n, seed, stream), ...] on the device:
    (x, y, z, offsets)."""
    import torch

    total = sum(int(s[1]) for s in sets)
    x, y, z = (torch.empty(max(total, 1), dtype=torch.float64, device=device) for _ in range(3))
    offs = device_generate(sets, x, y, z)
    return x, y, z, offs


def device_displace(x, y, z, sigma: float, seed: int, stream: int):
    """Move every particle of the float64 device tensors by N(0, sigma^2) per
    coordinate, in place (keyed by seed and stream; asynchronous)."""
    import torch

    n = x.numel()
    rc = _gpu_lib().wl_displace(x.data_ptr(), y.data_ptr(), z.data_ptr(), n, float(sigma), int(seed), int(stream),
                                torch.cuda.current_stream().cuda_stream)
    if rc != 0:
        raise RuntimeError("wl_displace failed")


def device_philox(counters: np.ndarray, key: tuple, device="cuda") -> np.ndarray:
    """Philox4x32-10 of (n, 4) uint32 counters under a 2-word key, on the device."""
    import torch

    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    ct = torch.from_numpy(c.view(np.int32)).to(device)
    out = torch.empty_like(ct)
    rc = _gpu_lib().wl_philox(ct.data_ptr(), c.shape[0], int(key[0]), int(key[1]), out.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    if rc != 0:
        raise RuntimeError("wl_philox failed")
    return out.cpu().numpy().view(np.uint32)
