"""Shared test helpers: device fixture logic and parameter mapping between the
HIP binding's SSIMConfig and the oracle's SSIMParams (configuration only, no
SSIM arithmetic)."""
import numpy as np
import pytest
import torch

MAP_TOL = 1e-5     # per map pixel, float32 path vs FP64 oracle
SCORE_TOL = 1e-6   # pooled scores


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this host")
    return torch.device("cuda:0")


def to_dev(a: np.ndarray, dev) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def oparams(cfg):
    import oracle as O
    return O.SSIMParams(window=cfg.window, k=cfg.k, sigma=cfg.sigma, C1=cfg.c1(), C2=cfg.c2(),
                        stride=cfg.stride, padding=cfg.padding)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """float32 -> nearest-even bfloat16 -> float64 (what the kernel reads)."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to(torch.float64).numpy()
