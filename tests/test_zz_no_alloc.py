"""hsdc_diffusion_solve_noalloc (the diffusion solve for callers that cannot
allocate device memory) against hsdc_diffusion_solve, through the C ABI: two
calls in a row on the library's static workspace, the second on a smaller
mesh, with a uniform and a per-node conductivity."""
import numpy as np
import pytest
import torch

import synthetic_inputs as si

pytestmark = pytest.mark.gpu

H = pytest.importorskip("paper_2405_19994_amd.hsdc")


def _case(dims, seed, per_node):
    rng = np.random.default_rng(seed)
    N = int(np.prod(dims))
    sig = None
    if per_node:
        sig = torch.tensor(np.exp(0.3 * rng.standard_normal(N)), dtype=torch.float64, device="cuda")
    prob = H.make_problem(dims, 0.025, (3.0, 1.0, 1.0)[:len(dims)] + (1.0,) * (3 - len(dims)), sig)
    b = torch.tensor(rng.uniform(-85.0, 30.0, N), dtype=torch.float64, device="cuda")
    x0 = b + torch.tensor(rng.standard_normal(N), dtype=torch.float64, device="cuda")
    return prob, b, x0


@pytest.mark.parametrize("per_node", [False, True])
def test_noalloc_solve_equals_allocating_solve(per_node):
    a = 0.05 * 0.3
    for dims, seed in (((300, 257), 1), ((61, 47), 2), ((20, 18, 9), 3)):
        prob, b, x0 = _case(dims, seed, per_node)
        x_ref, it_ref = H.diffusion_solve(prob, a, b, x0, rtol=1e-13, maxit=400)
        x = x0.clone()
        it = H.diffusion_solve_noalloc(prob, a, b, x, rtol=1e-13, maxit=400)
        torch.cuda.synchronize()
        assert it == it_ref
        err = float((x - x_ref).abs().max() / x_ref.abs().max())
        assert err < 1e-12, (dims, per_node, err)
        # the solve itself: ||b - A x|| <= rtol ||b||
        ax = x - a * H.apply_diffusion(prob, x)
        assert float(torch.linalg.vector_norm(b - ax)) <= 1e-13 * float(torch.linalg.vector_norm(b))


def test_noalloc_rejects_meshes_beyond_its_workspace():
    prob, b, x0 = _case((1024, 513), 4, False)
    with pytest.raises(H.HsdcError) as e:
        H.diffusion_solve_noalloc(prob, 0.01, b, x0)
    assert e.value.code == -1
