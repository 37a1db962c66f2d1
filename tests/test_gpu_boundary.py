"""Error paths of the boundary on the GPU: the binding refuses buffers the library would
overrun (too small, host memory, wrong dtype kind, not contiguous), and sap_set_gauge
refuses links that are not SU(3) (a U(3) link with det != 1, a non-unitary link, a NaN),
leaving the context without a gauge field until a valid one is set."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gu():
    import gpu_util
    return gpu_util


def test_binding_rejects_buffers_the_library_would_overrun(gu):
    import paper_0710_0066_amd as sap
    L = (4, 4, 2, 6)
    print("binding buffer checks", flush=True)
    ctx = gu.make_ctx(L, 2, 0.15, synth.gauge_field(L, 0.5, 11), max_rhs=2)
    good = ctx.new_field(2, sap.SAP_F32)
    bad = [good[:-1],                                          # one float short
           torch.zeros(good.numel(), dtype=torch.float32),    # host memory
           torch.zeros(good.numel(), dtype=torch.int32, device="cuda"),
           torch.zeros(2 * good.numel(), dtype=torch.float32, device="cuda")[::2]]   # strided
    for b in bad:
        with pytest.raises(sap.SapError) as e:
            sap.apply_Dslash_eo(ctx, b, good, 2, 0, sap.SAP_F32)
        assert e.value.code == sap.SAP_E_ARG
        with pytest.raises(sap.SapError) as e:
            sap.apply_M(ctx, good, b, 2, sap.SAP_F32)
        assert e.value.code == sap.SAP_E_ARG
    # a one-rhs FP64 field passed as two rhs, as FP64 where FP32 was allocated, momenta short
    one = ctx.new_field(1)
    with pytest.raises(sap.SapError):
        sap.solve_blocks(ctx, one, one.clone(), 2, 1, sap.SAP_ALL, sap.solve_opts())
    with pytest.raises(sap.SapError):
        sap.apply_M(ctx, ctx.new_field(2), good, 2, sap.SAP_F64)
    F = ctx.new_momenta()
    with pytest.raises(sap.SapError):
        sap.gauge_force(ctx, F[:-8], 1.0, 5.6)
    with pytest.raises(sap.SapError):
        ctx.set_gauge(torch.zeros(10, dtype=torch.complex128, device="cuda"))
    # the good buffers still work
    sap.apply_Dslash_eo(ctx, good, good.clone(), 2, 0, sap.SAP_F32)
    torch.cuda.synchronize()


def test_set_gauge_rejects_links_that_are_not_su3(gu):
    import paper_0710_0066_amd as sap
    L = (4, 4, 2, 6)
    print("SU(3) check", flush=True)
    U = synth.gauge_field(L, 0.5, 12)
    ctx = gu.make_ctx(L, 2, 0.15, U)            # SU(3): accepted
    assert 0.0 < sap.sap_plaquette(ctx) < 1.0
    phase = U.copy()
    phase[1, 2, 0, 3, 2] *= np.exp(0.3j)        # unitary, det = e^{0.9 i}
    scaled = U.copy()
    scaled[3, 0, 1, 5, 0] *= 1.001              # not unitary
    nan = U.copy()
    nan[0, 0, 0, 0, 1, 2, 2] = np.nan
    for bad in (phase, scaled, nan):
        with pytest.raises(sap.SapError) as e:
            ctx.set_gauge(gu.dev(bad))
        assert e.value.code == sap.SAP_E_ARG and "SU(3)" in str(e.value)
        with pytest.raises(sap.SapError) as e:      # no gauge field until a valid one is set
            sap.sap_plaquette(ctx)
        assert e.value.code == sap.SAP_E_STATE
    ctx.set_gauge(gu.dev(U))
    f = gu.to_sap(ctx, synth.gaussian_spinor(L, 13), 1)
    sap.apply_M(ctx, ctx.new_field(1), f, 1, sap.SAP_F64)
    torch.cuda.synchronize()
