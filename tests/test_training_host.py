"""CPU check of the training loss: the differentiable torch SSIM equals the
numpy definition (quality.ssim, pinned against a direct windowed sum)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_torch_ssim_equals_numpy_definition():
    from paper_2506_02774_amd import quality, training
    rng = np.random.default_rng(2)
    a = rng.random((3, 30, 41))
    b = np.clip(a + 0.1 * rng.standard_normal(a.shape), 0, 1)
    t = training.ssim(torch.from_numpy(a), torch.from_numpy(b)).item()
    assert abs(t - quality.ssim(a, b)) < 1e-12
    assert abs(training.ssim(torch.from_numpy(a), torch.from_numpy(a)).item() - 1.0) < 1e-12


def test_loss_gradient_flows():
    from paper_2506_02774_amd import training
    a = torch.rand(3, 20, 24, dtype=torch.float64, requires_grad=True)
    b = torch.rand(3, 20, 24, dtype=torch.float64)
    assert torch.autograd.gradcheck(lambda x: training.loss_l1_ssim(x, b), (a,), eps=1e-6, atol=1e-5)


def test_backward_refuses_a_stale_forward():
    """Two forwards on one Renderer before backward(): the first graph's
    backward must not silently take the second forward's saved state."""
    from paper_2506_02774_amd import VY_ERR_STATE, VoyagerError, training

    class StubRenderer:            # forward bookkeeping only; no GPU call is reached
        generation = 0

        def _render(self, params, cam):
            self.generation += 1
            return params["mean"].sum() * torch.ones(3, 2, 2)

    r = StubRenderer()
    p = {k: torch.zeros(4, 3, requires_grad=True) for k in training.PARAMS}
    a = training.GaussianRenderFn.apply(*[p[k] for k in training.PARAMS], r, None)
    b = training.GaussianRenderFn.apply(*[p[k] for k in training.PARAMS], r, None)
    with pytest.raises(VoyagerError) as e:
        a.sum().backward()
    assert e.value.code == VY_ERR_STATE
