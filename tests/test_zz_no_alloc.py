"""cstone_build_static (the build whose workspace is a fixed array inside the
library, for callers that cannot allocate) against cstone_build on the same
inputs, called through the C ABI: two calls in a row, the second smaller, so
the second runs on the first call's leftover scratch contents."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu

cs = pytest.importorskip("paper_2307_06345_amd")
lib = cs._lib

STATIC_BYTES = 64 << 20


def say(*a):
    print("[case]", *a, flush=True)


def outputs(n, cap, dev="cuda"):
    nn = cs.node_count(cap)
    return dict(P=torch.empty(max(n, 1), dtype=torch.int64, device=dev),
                perm=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                K=torch.empty(cap + 1, dtype=torch.int64, device=dev),
                N=torch.empty(cap, dtype=torch.int32, device=dev),
                NK=torch.empty(nn, dtype=torch.int64, device=dev),
                CO=torch.empty(nn, dtype=torch.int32, device=dev),
                LO=torch.empty(cs.LEVEL_OFFSETS, dtype=torch.int32, device=dev))


def run(static, s, cap):
    x, y, z = (cs.from_numpy(a, "cuda") for a in (s.x, s.y, s.z))
    o = outputs(s.n, cap)
    box = cs.Box.of(s.box)
    nl = ctypes.c_size_t(0)
    rounds = ctypes.c_uint32(0)
    stream = cs._stream()
    common = [cs._ptr(x), cs._ptr(y), cs._ptr(z), s.n, ctypes.byref(box), int(s.curve), int(s.n_crit),
              cs._ptr(o["P"]), cs._ptr(o["perm"]), cs._ptr(o["K"]), ctypes.byref(nl), cap, cs._ptr(o["N"]),
              cs._ptr(o["NK"]), cs._ptr(o["CO"]), cs._ptr(o["LO"]), 0, ctypes.byref(rounds)]
    if static:
        st = lib.cstone_build_static(*common, stream)
    else:
        ws = torch.empty(lib.cstone_build_workspace_bytes(s.n, cap), dtype=torch.uint8, device="cuda")
        st = lib.cstone_build(*common, cs._ptr(ws), ws.numel(), None, stream)
    torch.cuda.synchronize()
    assert st == 0, cs.STATUS.get(st, st)
    m = nl.value
    nn = cs.node_count(m)
    return dict(P=cs.to_numpy(o["P"][:s.n]), perm=cs.to_numpy(o["perm"][:s.n]), K=cs.to_numpy(o["K"][:m + 1]),
                N=cs.to_numpy(o["N"][:m]), NK=cs.to_numpy(o["NK"][:nn]), CO=cs.to_numpy(o["CO"][:nn]),
                LO=cs.to_numpy(o["LO"]), rounds=rounds.value)


def test_static_build_equals_the_build_twice_in_a_row():
    for kind, n, seed, curve, n_crit in (("plummer", 600001, 31, wl.HILBERT, 16), ("uniform", 40000, 32, wl.MORTON, 64)):
        s = wl.make_set(kind, n, seed, 0, curve, n_crit)
        cap = 8 * n // (n_crit + 1) + 64
        assert lib.cstone_build_workspace_bytes(n, cap) <= STATIC_BYTES
        say("static build", kind, n, n_crit)
        got = run(True, s, cap)
        ref = run(False, s, cap)
        for k in ref:
            assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), (kind, n, k)


def test_static_build_rejects_sizes_beyond_its_array():
    n = 1 << 23
    cap = 8 * n // 17
    assert lib.cstone_build_workspace_bytes(n, cap) > STATIC_BYTES
    box = cs.Box.of(((0.0, 0.0, 0.0), (1.0, 1.0, 1.0)))
    nl = ctypes.c_size_t(0)
    dummy = torch.empty(8, dtype=torch.int64, device="cuda")
    p = cs._ptr(dummy)
    st = lib.cstone_build_static(p, p, p, n, ctypes.byref(box), 1, 16, p, p, p, ctypes.byref(nl), cap, p, p, p, p, 0,
                                 None, cs._stream())
    assert cs.STATUS[st] == "INVALID_ARG"
