"""The evaluation entry point that allocates nothing
(dr_eval_logp_grad_noalloc) against the allocating one (dr_eval_logp_grad):
both run the same kernels on the same inputs, so every output is bit-equal.
Two calls in a row per mode, the second smaller (the fixed scratch buffer
keeps the first call's contents; the forward-only evaluator's counter is
cleared by the call itself), and the size limit is rejected on the host."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2605_08916_amd import dr, inputs  # noqa: E402


@pytest.fixture(scope="module")
def scene():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return dr.Scene(inputs.procedural_spheres(n_spheres=3, subdiv=3, width=128, height=128))


def _outputs(n, L, grad):
    d = 4 * (L - 1)
    nan = float("nan")
    return (torch.full((n, 3), nan, device="cuda"), torch.full((n,), nan, device="cuda"),
            torch.full((n, d), nan, device="cuda") if grad else None,
            torch.full((n, L - 1), -7, device="cuda", dtype=torch.int32))


@pytest.mark.parametrize("grad", [True, False])
def test_noalloc_matches_allocating_entry_point(scene, grad):
    L = 8
    d = 4 * (L - 1)
    for n in (60000, 3001):
        print(f"[no-alloc eval] L={L} n={n} grad={grad}", flush=True)
        u = torch.from_numpy(inputs.random_points(d, n, seed=n)).cuda()
        f0, lp0, g0, r0 = scene.eval_logp_grad(L, u, grad=grad, rec=True)
        f1, lp1, g1, r1 = _outputs(n, L, grad)
        scene.eval_logp_grad_into(L, u, f1, lp1, g1, r1)
        torch.cuda.synchronize()
        assert torch.equal(f0, f1) and torch.equal(lp0, lp1) and torch.equal(r0, r1)
        if grad:
            assert torch.equal(g0, g1)
        assert bool(torch.isfinite(f1).all())


def test_noalloc_rejects_inputs_beyond_its_scratch(scene):
    L = 8
    n = (16 << 20) // (4 * (L - 1)) + 1   # one point more than the 16 MiB of path records hold
    u = torch.zeros((n, 4 * (L - 1)), device="cuda")
    f, lp, g, r = _outputs(n, L, True)
    with pytest.raises(dr.DrError) as e:
        scene.eval_logp_grad_into(L, u, f, lp, g, r)
    assert e.value.status == dr.DR_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool(torch.isnan(f).all())   # nothing ran
    # forward-only needs no per-point scratch: the same size is accepted
    f2, lp2, _, r2 = _outputs(n, L, False)
    scene.eval_logp_grad_into(L, u, f2, lp2, None, r2)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(f2).all())
