"""The outer calibration loop (Sec. IV-B) on the stand-in model: sigmoid-reparametrised
multipliers, Adam from the midpoint of the range, the unidirectional Chamfer loss through the GPU
path, best-loss selection.  It must recover known multipliers from a noisy synthetic target."""
import json

import numpy as np
import pytest

from gpu_helpers import gpu, say, torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_calibration_recovers_multipliers(precision):
    p = gpu()
    from paper_2204_03139_amd import calibrate as cal
    say(f"[calibrate] precision={precision}")
    model = cal.StandInCloth(T=10)
    w_true = (2.0, 6.0)
    obs = cal.synthetic_target(model, w_true, 2048)
    out = cal.calibrate(model, obs, 2048, iters=150, precision=precision)
    say(f"[calibrate] {json.dumps(dict(w=out['w'], loss=out['loss']))}")
    # the loss at the true multipliers (same sampling seed) bounds what the search can reach
    with torch.no_grad():
        v = model(torch.tensor(w_true, dtype=torch.float64, device="cuda"))
        l_true = p.diffcloud_loss(v, model.faces, obs, 2048, seed=1000, precision=precision,
                                  reduction=1).item()
    first = out["history"][0][0]
    assert out["loss"] <= 1.05 * l_true and out["loss"] < 0.5 * first
    assert abs(out["w"][0] - w_true[0]) <= 0.1 * w_true[0]
    assert abs(out["w"][1] - w_true[1]) <= 0.1 * w_true[1]
    # the stand-in's gradient path: autograd through the model matches a central difference
    s = torch.tensor([0.3, -0.2], dtype=torch.float64, device="cuda", requires_grad=True)
    loss = p.diffcloud_loss(model(cal.multipliers(s)), model.faces, obs, 2048, seed=5,
                            precision=precision, reduction=1)
    loss.backward()
    g = s.grad.cpu().numpy()
    assert np.all(np.isfinite(g)) and np.any(g != 0)
