"""The allocation-free force profile (sap_force_profile_noalloc) against the allocating
entry point sap_force_profile, through the C ABI: two calls in a row on one GPU, the
second on a smaller lattice, so that the second reuses the fixed partial-sum array the
first left filled. The two entry points run the same kernels in the same order, so the
profiles must agree bit for bit; both are also held to the oracle's profile."""
import numpy as np
import pytest
import torch

import synth
from oracle import forces

pytestmark = pytest.mark.gpu


def _profile_pair(sap, gu, L, l0, seed):
    ctx = gu.make_ctx(L, l0, 0.15, synth.gauge_field(L, 0.5, seed))
    p = synth.gaussian_momenta(L, seed + 1)
    F = ctx.new_momenta()
    ctx.pack_momenta(F, gu.dev(p))
    ref = np.array(sap.sap_force_profile(ctx, F))
    prof = torch.full((2 * L[0],), float("nan"), dtype=torch.float64, device="cuda")
    sap.sap_force_profile_noalloc(ctx, F, prof)
    torch.cuda.synchronize()
    got = prof.cpu().numpy().reshape(2, L[0])
    return got, ref, forces.force_profile(p)


def test_force_profile_noalloc_matches_allocating_entry():
    import gpu_util as gu
    import paper_0710_0066_amd as sap
    assert sap.sap_force_profile_noalloc_max() == 1 << 18
    # first a lattice with three 128-site chunks per slice (the last one ragged), then a
    # smaller one with a single chunk
    for L, l0, seed in [((16, 8, 8, 12), 4, 301), ((6, 2, 4, 6), 3, 303)]:
        print(f"force profile noalloc L={L}", flush=True)
        got, ref, orc = _profile_pair(sap, gu, L, l0, seed)
        assert np.array_equal(got, ref), (L, np.max(np.abs(got - ref)))
        assert np.max(np.abs(got - orc)) <= 1e-13 * np.max(np.abs(orc)), L


def test_force_profile_noalloc_rejects_null_pointers():
    """The library's own host-side check (called past the binding, which refuses None)."""
    import ctypes
    import gpu_util as gu
    import paper_0710_0066_amd as sap
    L = (6, 2, 4, 6)
    ctx = gu.make_ctx(L, 3, 0.15, synth.gauge_field(L, 0.5, 305))
    F = ctx.new_momenta()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = sap._lib.sap_force_profile_noalloc(ctx.ptr, ctypes.c_void_p(F.data_ptr()), None, stream)
    assert rc == sap.SAP_E_ARG
    rc = sap._lib.sap_force_profile_noalloc(ctx.ptr, None, ctypes.c_void_p(F.data_ptr()), stream)
    assert rc == sap.SAP_E_ARG
    with pytest.raises(sap.SapError) as e:
        sap.sap_force_profile_noalloc(ctx, F, None)
    assert e.value.code == sap.SAP_E_ARG
