"""The autograd loss refuses operands the loss entry points cannot take
(wrong dtype, wrong device, wrong shape) before any library call: checked on
the CPU with a stand-in problem whose handle is never used."""

import pytest
import torch

from paper_1510_05237_amd import NMFLoss


class _Stub:
    h = None
    n, m, k = 7, 5, 3
    torch_dtype = torch.float32
    device = torch.device("cuda:0")
    stream = None


def _expect(exc, U, V):
    with pytest.raises(exc):
        NMFLoss.apply(_Stub(), U, V)


def test_loss_refuses_host_tensors():
    _expect(ValueError, torch.zeros(7, 3), torch.zeros(5, 3))


def test_loss_refuses_wrong_dtype():
    _expect(TypeError, torch.zeros(7, 3, dtype=torch.float64), torch.zeros(5, 3))


def test_loss_refuses_wrong_shapes():
    s = _Stub()
    s.device = torch.device("cpu")  # so that only the shape check can fail
    for U, V in ((torch.zeros(6, 3), torch.zeros(5, 3)), (torch.zeros(7, 3), torch.zeros(5, 4)),
                 (torch.zeros(7, 4), torch.zeros(5, 4))):
        with pytest.raises(ValueError):
            NMFLoss.apply(s, U, V)


def test_loss_refuses_non_tensors():
    import numpy as np

    _expect(TypeError, np.zeros((7, 3), np.float32), torch.zeros(5, 3))
