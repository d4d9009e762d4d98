"""Helpers shared by the GPU tests (device buffers, seeded inputs, tolerances)."""
from __future__ import annotations

import numpy as np


def to_dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def map_tolerance(p_oracle: np.ndarray, t_oracle: np.ndarray, eps: float,
                  template_exact: bool = False) -> np.ndarray:
    """Per-window bound on the Bhattacharyya error implied by a histogram error.

    If every normalised bin of the window and of the template is within
    ``eps`` of the oracle's, then with |sqrt(a') - sqrt(a)| <= d(a) =
    min(sqrt(eps), eps / sqrt(a)):
      |sqrt(p' t') - sqrt(p t)| <= d(p) (sqrt(t) + d(t)) + sqrt(p) d(t).
    ``template_exact`` drops the template's share (the oracle's template is fed).
    p_oracle: [n, B]; t_oracle: [B].  Returns [n].
    """
    def d(a):
        a = np.maximum(a, 0.0)
        with np.errstate(divide="ignore"):
            return np.minimum(np.sqrt(eps), np.where(a > 0, eps / np.sqrt(a), np.inf))

    dp = d(p_oracle)
    st = np.sqrt(np.maximum(t_oracle, 0.0))[None, :]
    if template_exact:
        return (dp * st).sum(1)
    dt = d(t_oracle)[None, :]
    return (dp * (st + dt) + np.sqrt(np.maximum(p_oracle, 0.0)) * dt).sum(1)
