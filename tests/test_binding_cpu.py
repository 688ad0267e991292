"""The Python binding rejects malformed output and gradient tensors before it
hands any pointer to the library (no GPU and no library call needed)."""
import pytest
import torch

from paper_2403_19854_amd import fcrkpm


def _problem(nn=8):
    # a Problem shell on the CPU: enough for the argument checks, which run
    # before the first library call
    p = fcrkpm.Problem.__new__(fcrkpm.Problem)
    p.device = torch.device("cpu")
    p.nn = nn
    p.shape = (2, 2, 2)
    p._h = None
    return p


@pytest.mark.parametrize("bad", [
    torch.empty(8, dtype=torch.float32),            # wrong dtype for an FP64 apply
    torch.empty(7, dtype=torch.float64),            # too few values
    torch.empty(16, dtype=torch.float64),           # too many values
    torch.empty(16, dtype=torch.float64)[::2],      # not contiguous
])
def test_apply_rejects_bad_out(bad):
    p = _problem()
    with pytest.raises(ValueError):
        p.apply("K", torch.zeros(8, dtype=torch.float64), out=bad)


def test_apply_rejects_out_of_other_precision_fp32_input():
    p = _problem()
    with pytest.raises(ValueError):
        p.apply("K", torch.zeros(2, 8, dtype=torch.float32), out=torch.empty(2, 8, dtype=torch.float64))


@pytest.mark.parametrize("fn", ["nonlinear_force", "gradient_force"])
def test_forces_reject_bad_out(fn):
    p = _problem()
    d = torch.zeros(2, 8, dtype=torch.float64)
    for bad in (torch.empty(8, dtype=torch.float64), torch.empty(2, 8, dtype=torch.float32),
                torch.empty(2, 16, dtype=torch.float64)[:, ::2]):
        with pytest.raises(ValueError):
            getattr(p, fn)(d, 1.0, out=bad)


def test_adjoint_rejects_partial_fields():
    p = _problem()
    with pytest.raises(ValueError):
        p.adjoint(torch.zeros(12, dtype=torch.float64))


def test_input_not_whole_fields():
    p = _problem()
    with pytest.raises(ValueError):
        p.apply("K", torch.zeros(12, dtype=torch.float64))
    with pytest.raises(ValueError):
        p.nonlinear_force(torch.zeros(5, dtype=torch.float64), 1.0)
