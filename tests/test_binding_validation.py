"""The binding validates every caller buffer before its pointer reaches the
library (a float32 or wrongly shaped factor would otherwise be read past its
end on the device).  CPU only: the checks run before any library call, so a
context object with the shape attributes set is enough, and the library
function is replaced by one that fails the test if reached."""
import numpy as np
import pytest
import torch

import paper_2112_03985_amd as jk


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError("library function %s reached past validation" % name)


@pytest.fixture
def ctx(monkeypatch):
    monkeypatch.setattr(jk, "lib", lambda: _NoLib())
    c = object.__new__(jk.JkCals)
    c.dims = [4, 5, 6]
    c.N = 3
    c.C = 7
    c.K = 2
    c.device = torch.device("cpu")
    c.ctx = None
    return c


def test_set_factors_rejects_float32(ctx):
    with pytest.raises(TypeError):
        ctx.set_factors(0, torch.zeros((4, 7), dtype=torch.float32))


def test_set_factors_rejects_wrong_shape(ctx):
    with pytest.raises(ValueError):
        ctx.set_factors(1, torch.zeros((4, 7), dtype=torch.float64))
    with pytest.raises(ValueError):
        ctx.set_factors(0, torch.zeros((4, 8), dtype=torch.float64))


def test_set_factors_rejects_non_contiguous(ctx):
    with pytest.raises(ValueError):
        ctx.set_factors(0, torch.zeros((7, 4), dtype=torch.float64).t())


def test_set_factors_rejects_host_tensor_and_bad_lambda(ctx):
    with pytest.raises(ValueError):
        ctx.set_factors(0, torch.zeros((4, 7), dtype=torch.float64))
    with pytest.raises(TypeError):
        ctx.set_factors(0, torch.zeros((4, 7), dtype=torch.float64), torch.ones(7, dtype=torch.float32))


def test_mode_out_of_range(ctx):
    for bad in (-1, 3):
        with pytest.raises(ValueError):
            ctx.set_factors(bad, torch.zeros((4, 7), dtype=torch.float64))


def test_output_buffers_are_checked(ctx):
    with pytest.raises(ValueError):
        ctx.mttkrp(2, out=torch.zeros((5, 7), dtype=torch.float64))
    with pytest.raises(TypeError):
        ctx.get_grad(0, out=torch.zeros((4, 7), dtype=torch.float32))
    with pytest.raises(ValueError):
        ctx.get_grad(0, weights=torch.ones(3, dtype=torch.float64),
                     out=torch.zeros((4, 7), dtype=torch.float64))
    with pytest.raises(ValueError):
        ctx.loss_grad(torch.zeros(3, dtype=torch.float64))
    with pytest.raises(ValueError):
        ctx.refine(2, torch.zeros(1, dtype=torch.float64))
    with pytest.raises(ValueError):
        ctx.sweep(1, torch.zeros(5, dtype=torch.float64))
    with pytest.raises(ValueError):
        ctx.scale_columns(torch.zeros((4, 6), dtype=torch.float64))


def test_remove_slice_checks_its_buffers(monkeypatch):
    monkeypatch.setattr(jk, "lib", lambda: _NoLib())
    T = torch.zeros(4 * 5 * 6, dtype=torch.float64)
    with pytest.raises(ValueError):
        jk.jk_cals_remove_slice(T, [4, 5, 6], 0, 1)       # host tensor
    with pytest.raises(TypeError):
        jk.jk_cals_remove_slice(T.to(torch.int32), [4, 5, 6], 0, 1)
