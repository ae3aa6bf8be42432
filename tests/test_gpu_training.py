"""GPU checks of the autograd path (training.Renderer over vy_render_backward):
its gradients equal the C-ABI backward's for the same dL/dimage, and a few
Adam steps on L1 + 0.2 (1 - SSIM) pull perturbed Gaussians towards a target
image rendered from the original ones."""
import numpy as np
import pytest

import scenegen

from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

W, H = 64, 48


@pytest.fixture(scope="module")
def setup():
    vy = require_gpu()
    import torch
    from paper_2506_02774_amd import training
    leaves = scenegen.random_gaussians(600, 31, W, H, depth_range=(2.0, 12.0), scale_range=(-2.5, -1.0))
    host = scenegen.build_hierarchy(dict(mean=leaves.mean, log_scale=leaves.log_scale, quat=leaves.quat,
                                         opacity_logit=leaves.opacity_logit, sh=leaves.sh))
    cam = scenegen.identity_camera(W, H)
    return vy, torch, training, host, cam


def test_autograd_equals_c_abi(setup):
    vy, torch, training, host, cam = setup
    r = training.Renderer(host, W, H, tau=0.0, bg=(0.2, 0.1, 0.0))
    params = r.parameters_from(host)
    w = torch.randn(3, H, W, device="cuda", generator=torch.Generator(device="cuda").manual_seed(0))
    img = r(params, cam)
    (img * w).sum().backward()
    g = vy.vy_render_backward(r.scene, r.cut, cam, r.ctx, w.contiguous(), quat_raw=params["quat"].detach())
    for k in training.PARAMS:
        a, b = params[k].grad, g[k].reshape(params[k].shape)
        scale = max(1e-6, float(b.abs().max()))
        assert float((a - b).abs().max()) <= 1e-5 * scale, k
        assert float(b.abs().max()) > 0, k


def test_adam_steps_reduce_l1_ssim(setup):
    vy, torch, training, host, cam = setup
    r = training.Renderer(host, W, H, tau=0.0)
    target = r(r.parameters_from(host), cam).detach()
    params = r.parameters_from(host)
    gen = torch.Generator(device="cuda").manual_seed(1)
    leaf = torch.as_tensor(host.child_count == 0, device="cuda")
    with torch.no_grad():
        params["sh"][leaf] += 0.15 * torch.randn(params["sh"][leaf].shape, device="cuda", generator=gen)
        params["opacity_logit"][leaf] += 0.5 * torch.randn(params["opacity_logit"][leaf].shape, device="cuda",
                                                           generator=gen)
    opt = torch.optim.Adam([params[k] for k in training.PARAMS], lr=0.01)
    losses = []
    for step in range(40):
        opt.zero_grad()
        loss = training.loss_l1_ssim(r(params, cam), target)
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    print("loss:", [round(x, 5) for x in losses[::8]], losses[-1], flush=True)
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.5 * losses[0]


def test_backward_after_a_second_forward_is_refused(setup):
    vy, torch, training, host, cam = setup
    r = training.Renderer(host, W, H, tau=0.0)
    params = r.parameters_from(host)
    first = r(params, cam)
    second = r(params, cam)
    with pytest.raises(vy.VoyagerError) as e:
        first.sum().backward()
    assert e.value.code == vy.VY_ERR_STATE
    second.sum().backward()                       # the latest forward still differentiates
    assert float(params["sh"].grad.abs().max()) > 0


def test_update_gaussians_equals_a_fresh_upload(setup):
    """vy_scene_update_gaussians over the same tree renders bitwise what a
    fresh upload of the new parameters renders; a backward of a frame
    rendered before the update is refused."""
    vy, torch, training, host, cam = setup
    r = training.Renderer(host, W, H, tau=0.0)
    params = r.parameters_from(host)
    img0 = r(params, cam).detach().clone()
    gen = torch.Generator(device="cuda").manual_seed(9)
    new = {k: (v.detach() + 0.05 * torch.randn(v.shape, device="cuda", generator=gen)).contiguous()
           for k, v in params.items()}
    sc = vy.Scene.from_tensors(r.tree, new)
    cut = vy.vy_lod_cut(sc, cam, 0.0)
    ctx = vy.RenderContext(sc.n, W, H, 1 << 22)
    ref = vy.vy_render(sc, cut, cam, ctx, alpha_filter=True)
    w = torch.ones((3, H, W), device="cuda")
    r.scene.update_gaussians(new)                        # after the forward of img0: its backward is refused
    with pytest.raises(vy.VoyagerError) as e:
        vy.vy_render_backward(r.scene, r.cut, cam, r.ctx, w)
    assert e.value.code == vy.VY_ERR_STATE
    got = vy.vy_render(r.scene, r.cut, cam, r.ctx, alpha_filter=True)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32))
    assert not torch.equal(got, img0)
