"""Helpers shared by the GPU tests (not collected)."""
import numpy as np
import pytest

import scenegen


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_02774_amd as vy
    vy.lib()      # raises if the library is missing: no fallback
    return vy


def image_parity(gpu_img, ref, max_abs=2e-3, mean_abs=1e-4):
    """Compare a GPU image with the oracle image (the parity bar: max abs error
    2e-3 per channel over the pixels that are not ambiguous, mean abs error
    1e-4 over all pixels). Pixels the oracle did not render (NaN, when it
    rendered a subset of tiles) are left out."""
    g = np.asarray(gpu_img, np.float64)
    r = ref["image"]
    done = ~np.isnan(r[0])
    amb = ref["ambiguous"] & done
    err = np.abs(g - np.nan_to_num(r))[:, done]
    ok_pix = ~amb[done]
    mx = float(err[:, ok_pix].max()) if ok_pix.any() else 0.0
    mean = float(err.mean()) if err.size else 0.0
    return dict(max_abs=mx, mean_abs=mean, ambiguous=int(amb.sum()), n_pix=int(done.sum()),
                ok=(mx <= max_abs and mean <= mean_abs))


def random_cameras(cfg, n, seed, width=256, height=192):
    rng = np.random.default_rng(seed)
    cams = []
    for _ in range(n):
        p = rng.uniform(-0.3, 0.3, 2) * cfg.extent
        cams.append(scenegen.look_camera([p[0], p[1], rng.uniform(1.0, 60.0)], rng.uniform(0, 2 * np.pi),
                                         rng.uniform(-0.6, 0.2), width, height))
    return cams
