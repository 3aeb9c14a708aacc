"""The warm-start network's wrappers refuse tensors the kernels would misread
(host memory, wrong dtype, shape or layout) before any device call (no GPU)."""
import pytest
import torch

from paper_2609_31347_amd import warmstart as W


def _net():
    net = W.ConvNet.__new__(W.ConvNet)         # no weights: the checks come first
    net.layers = W.LAYERS
    return net


def test_host_tensors_are_refused():
    with pytest.raises(TypeError):
        W.to_bf16(torch.zeros(4))
    with pytest.raises(TypeError):
        W.mse(torch.zeros(1, 2, 3, 3), torch.zeros(1, 2, 3, 3), torch.ones(1, 3, 3))
    with pytest.raises(TypeError):
        _net().forward(torch.zeros(1, W.LAYERS[0][0], 4, 4, dtype=torch.bfloat16))


def test_need_checks_dtype_layout_and_shape():
    class Fake:                                  # a stand-in that claims to be a CUDA tensor
        is_cuda = True

    t = torch.zeros(2, 3, 4, 5, dtype=torch.float32)
    with pytest.raises(TypeError):
        W._need(t, torch.float32, t.shape, "x")              # host tensor
    with pytest.raises(TypeError):
        W._need(Fake(), torch.float32, (1,), "x")            # not a tensor


def test_backward_needs_a_forward():
    with pytest.raises(RuntimeError, match="forward"):
        _net().backward(torch.zeros(1, 2, 4, 4))


def test_first_layer_takes_the_seven_input_channels():
    assert W.LAYERS[0][0] == 7 and W.LAYERS[-1][1] == 2
