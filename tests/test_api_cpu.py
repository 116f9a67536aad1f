"""Host-side checks of the torch-facing call (no GPU): it refuses host
tensors and mismatched shapes before reaching the library."""
import pytest
import torch

from paper_0707_2347_amd import api


def test_refuses_host_tensors_and_bad_shapes():
    A = torch.zeros((4, 5), dtype=torch.float64)
    B = torch.zeros((5, 3), dtype=torch.float64)
    with pytest.raises(ValueError):
        api.mod_p_matmul(A, B, p=65521)
    with pytest.raises(ValueError):
        api._ld(torch.zeros(3), "A")
    assert api._ld(torch.zeros((4, 6))[:, :5], "A") == 6
    with pytest.raises(ValueError):
        api._ld(torch.zeros((6, 4)).t(), "A")
