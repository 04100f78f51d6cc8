"""fvim_operator_apply_noalloc (the operator entry point that allocates
nothing) against fvim_operator_apply, through the C ABI: two calls in a row
on one device, the second on a smaller grid, in float64 and in the
float32 mode, and the rejection of an application larger than the scratch."""
import numpy as np
import pytest
import torch

from paper_1811_11558_amd import Context, FvimError, NOALLOC_BYTES
from paper_1811_11558_amd import binding as b
from synth import filtered_eigenstrain, filtered_traction, grid_dict

pytestmark = pytest.mark.gpu

# the float64 bar of the operator tests (relative L2 per output)
TOL = 1e-11


def _rel(a, r):
    a = a.double().cpu().numpy()
    r = r.double().cpu().numpy()
    return np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300)


def _apply_both(g, precision, seed, want=("strain", "surf_u3")):
    ctx = Context(g, 1.0, 0.3, precision=precision)
    eps = torch.from_numpy(filtered_eigenstrain(g, seed=seed)).cuda()
    t = torch.from_numpy(filtered_traction(g, seed=seed + 1)).cuda()
    ref = ctx.operator_apply(eps, t, want=want)
    shapes = {"strain": ctx.tensor_shape, "stress": ctx.tensor_shape, "disp": ctx.vector_shape,
              "surf_u3": ctx.surface_shape}
    out = {k: torch.full(shapes[k], float("nan"), dtype=torch.float64, device="cuda") for k in want}
    ctx.operator_apply_noalloc(eps, t, out=out)
    torch.cuda.synchronize()
    return ctx, eps, t, ref, out


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_noalloc_matches_operator_apply_on_two_calls_second_smaller(precision):
    print("noalloc: %s, 128x128x32 then 64x32x9" % precision, flush=True)
    big = grid_dict(128, 128, 32, lz=0.25)
    small = grid_dict(64, 32, 9, lx=1.3, ly=0.7, lz=0.2)
    c1, _, _, ref1, out1 = _apply_both(big, precision, seed=5, want=("strain", "stress", "surf_u3"))
    for k in ref1:
        assert torch.isfinite(out1[k]).all(), k
        assert _rel(out1[k], ref1[k]) <= TOL, (k, _rel(out1[k], ref1[k]))
    # second call, smaller grid: the scratch still holds the first call's data
    c2, eps2, t2, ref2, out2 = _apply_both(small, precision, seed=9, want=("strain", "disp", "surf_u3"))
    for k in ref2:
        assert torch.isfinite(out2[k]).all(), k
        assert _rel(out2[k], ref2[k]) <= TOL, (k, _rel(out2[k], ref2[k]))
    if precision == "fp64":
        from oracle import operators as ora
        o = ora.apply(small, 1.0, 0.3, eps_p=eps2.cpu().numpy(), traction=t2.cpu().numpy())
        for k in ("strain", "disp", "surf_u3"):
            assert _rel(out2[k], torch.from_numpy(o[k])) <= TOL, k
    c1.close()
    c2.close()


def test_noalloc_rejects_an_application_larger_than_the_scratch():
    print("noalloc: 128x128x64 strain+stress+disp (too large)", flush=True)
    g = grid_dict(128, 128, 64, lz=0.25)
    ctx = Context(g, 1.0, 0.3)
    eps = torch.zeros(ctx.tensor_shape, dtype=torch.float64, device="cuda")
    out = {"strain": torch.empty(ctx.tensor_shape, dtype=torch.float64, device="cuda"),
           "stress": torch.empty(ctx.tensor_shape, dtype=torch.float64, device="cuda"),
           "disp": torch.empty(ctx.vector_shape, dtype=torch.float64, device="cuda")}
    with pytest.raises(FvimError) as ei:
        ctx.operator_apply_noalloc(eps, None, out=out)
    assert ei.value.code == b.FVIM_EINVAL
    assert "scratch" in str(ei.value)
    assert NOALLOC_BYTES == 128 << 20
    ctx.close()
