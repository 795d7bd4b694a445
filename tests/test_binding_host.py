"""Argument checks of the Python binding (no GPU): tensors the library reads
or writes through raw device pointers are rejected before any library call
when their type, size or device is wrong."""
import pytest
import torch

from paper_2010_11130_amd.api import _vec


def test_wrong_dtype_rejected():
    with pytest.raises(ValueError, match="floating-point"):
        _vec(torch.zeros(5, dtype=torch.int32), 5, "rhs")
    with pytest.raises(ValueError, match="float64"):
        _vec(torch.zeros(5, dtype=torch.float32), 5, "out", out=True)


def test_wrong_length_rejected():
    with pytest.raises(ValueError, match="expected 6 values"):
        _vec(torch.zeros(5, dtype=torch.float64), 6, "rhs")
    with pytest.raises(ValueError, match="expected 6 values"):
        _vec(torch.zeros(7, dtype=torch.float64), 6, "out", out=True)


def test_host_tensor_rejected():
    with pytest.raises(ValueError, match="device memory"):
        _vec(torch.zeros(5, dtype=torch.float64), 5, "g")


def test_none_passes_through():
    assert _vec(None, 5, "rhs") is None
