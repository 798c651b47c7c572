"""The order network's training checkpoint (weights, both Adam moment
estimates, schedule stage and step, loss history) round-trips through its file
exactly, and a file of the wrong size is refused."""
import numpy as np
import pytest

from paper_2009_00767_amd import FMM_MLP_NPARAM, order_model


def test_checkpoint_round_trip(tmp_path):
    rng = np.random.default_rng(5)
    w, m1, m2 = (rng.normal(size=FMM_MLP_NPARAM).astype(np.float32) for _ in range(3))
    path = str(tmp_path / "ck.npz")
    order_model.save_checkpoint(path, w, m1, m2, 2, 137, [0.5, 0.25])
    st = order_model.load_checkpoint(path)
    np.testing.assert_array_equal(st["w"], w)
    np.testing.assert_array_equal(st["m1"], m1)
    np.testing.assert_array_equal(st["m2"], m2)
    assert (st["stage"], st["step"]) == (2, 137)
    np.testing.assert_array_equal(st["losses"], np.float32([0.5, 0.25]))
    order_model.save_checkpoint(path, w[:10], m1, m2, 0, 0, [])
    with pytest.raises(ValueError):
        order_model.load_checkpoint(path)
