"""CPU checks of the torch-side helpers: the signed-scale activation and the
mapping from the paper's signed scales to (sigma, lambda)."""
import numpy as np
import torch

from paper_2411_16392_amd import render as R


def test_signed_scale_activation_and_gradient():
    # s = tanh(t) exp(x): sign from t, magnitude from x, differentiable through 0
    x = torch.tensor([0.3, -1.2, 2.0, 0.0], dtype=torch.float64, requires_grad=True)
    t = torch.tensor([1.5, -0.7, 0.0, -3.0], dtype=torch.float64, requires_grad=True)
    s = R.signed_scale(x, t)
    assert torch.allclose(s, torch.tanh(t) * torch.exp(x))
    assert torch.all(torch.sign(s[:2]) == torch.sign(t[:2]))
    assert s[2] == 0.0
    assert torch.autograd.gradcheck(R.signed_scale, (x, t))


def test_signed_scales_map_onto_the_explicit_paraboloid():
    # f = sign(s1)/s1^2 x^2 + sign(s2)/s2^2 y^2 - z/s3 = 0 (implicit form, Sec. 3.2)
    # is z = lambda1 x^2 + lambda2 y^2 with lambda_i = sign(s_i) s3 / s_i^2
    rng = np.random.default_rng(3)
    s1 = torch.tensor(rng.uniform(0.1, 1.0, 50) * rng.choice([-1, 1], 50), dtype=torch.float64)
    s2 = torch.tensor(rng.uniform(0.1, 1.0, 50) * rng.choice([-1, 1], 50), dtype=torch.float64)
    s3 = torch.tensor(rng.uniform(0.1, 2.0, 50), dtype=torch.float64)
    sigma, lam = R.signed_scale_to_params(s1, s2, s3)
    assert torch.all(sigma > 0)
    x = torch.tensor(rng.uniform(-1, 1, 50), dtype=torch.float64)
    y = torch.tensor(rng.uniform(-1, 1, 50), dtype=torch.float64)
    z = lam[:, 0] * x * x + lam[:, 1] * y * y
    f = torch.sign(s1) / s1 ** 2 * x * x + torch.sign(s2) / s2 ** 2 * y * y - z / s3
    assert torch.max(torch.abs(f)) < 1e-12
