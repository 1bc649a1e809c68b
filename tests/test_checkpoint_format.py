"""Checkpoint files on the host: the geometry metadata round trip, and files of the wrong kind are
refused before anything is created."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
safetensors_torch = pytest.importorskip("safetensors.torch")

import synth  # noqa: E402
from paper_2206_15117_amd import checkpoint  # noqa: E402


def test_geometry_metadata_round_trip():
    g = synth.config2().geom
    back = checkpoint._geometry_from(checkpoint._geometry_meta(g))
    assert (back.n, back.cell, back.os, back.aa_support, back.mk) == (g.n, g.cell, g.os, g.aa_support, g.mk)
    assert np.array_equal(back.w_planes, g.w_planes) and back.w_planes.dtype == np.float64
    assert np.array_equal(back.support, g.support) and np.array_equal(back.tile, g.tile)
    assert back.nplanes == g.nplanes and back.fov == g.fov


def test_wrong_file_kind_is_refused(tmp_path):
    path = str(tmp_path / "x.safetensors")
    safetensors_torch.save_file({"table": torch.zeros(4, 2)}, path, metadata={"format": checkpoint.KERNELS_FORMAT})
    with pytest.raises(ValueError, match="expected 'polgrid-mlp-1'"):
        checkpoint.load_network(path)
    other = str(tmp_path / "y.safetensors")
    safetensors_torch.save_file({"w.0": torch.zeros(2, 2)}, other)
    with pytest.raises(ValueError, match="expected 'polgrid-kernels-1'"):
        checkpoint.load_kernels(other)
