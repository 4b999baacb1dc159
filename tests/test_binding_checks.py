"""The Python binding refuses buffers that do not match what the C ABI will read or
write (length, dtype, layout, memory kind) before any library call."""
import numpy as np
import pytest
import torch

from paper_2007_02082_amd import _lib


def _bare_solver(n_u=10, n_p=10, M=2):
    """A Solver object without a context: only the argument checks can run."""
    s = _lib.Solver.__new__(_lib.Solver)
    s._h, s._stream, s._dev = None, None, None
    s.n_u, s.n_p, s.M = n_u, n_p, M
    return s


@pytest.mark.parametrize("u, p", [
    (np.zeros(29), np.zeros(10)),                                   # short u
    (np.zeros(30), np.zeros(11)),                                   # long p
    (torch.zeros(30, dtype=torch.float32), torch.zeros(10, dtype=torch.float64)),
    (torch.zeros(30, dtype=torch.float64), torch.zeros(10, dtype=torch.float32)),
    (torch.zeros(60, dtype=torch.float64)[::2], torch.zeros(10, dtype=torch.float64)),  # strided
    (torch.zeros(29, dtype=torch.float64), torch.zeros(10, dtype=torch.float64)),
    ([0.0] * 30, np.zeros(10)),                                     # not an array
])
def test_set_state_rejects_bad_buffers(u, p):
    s = _bare_solver()
    with pytest.raises(ValueError):
        s.set_state(u, p, 0.0)


def test_get_state_device_rejects_host_and_short_buffers():
    s = _bare_solver()
    with pytest.raises(ValueError):
        s.get_state_device(torch.zeros(30, dtype=torch.float64), torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError):
        s.get_state_device(torch.zeros(30, dtype=torch.float32), torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError):
        s.get_state_device(np.zeros(30), np.zeros(10))


def test_set_points_apply_and_wall_shear_check_lengths():
    s = _bare_solver()
    with pytest.raises(ValueError):
        s.set_points(np.zeros((3, 3)))                              # M = 2 points expected
    with pytest.raises(ValueError):
        s.set_points(np.zeros((2, 3)), np.zeros((1, 3)))             # short U_B
    with pytest.raises(ValueError):
        s.set_points(torch.zeros(6, dtype=torch.float32))
    with pytest.raises(ValueError):
        s.apply(_lib.OP_GRAD, np.zeros(30))                          # gradient takes n_p values
    with pytest.raises(ValueError):
        s.apply(_lib.OP_INTERP, np.zeros(6))                         # interpolation takes 3 n_u
    with pytest.raises(ValueError):
        s.wall_shear(np.zeros((3, 3)))
