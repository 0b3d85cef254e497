"""Seeded QSGS mask generator: exact porosity, percolation, determinism."""
import os

import numpy as np
import pytest
from scipy import ndimage

from paper_1609_09685_amd import qsgs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_2d():
    out = []
    with open(os.path.join(GOLDEN, "paper_values.txt")) as fh:
        for line in fh:
            t = line.split("#")[0].split()
            if t and t[0] == "2d":
                out.append((int(t[1]), int(t[2]), float(t[3])))
    return out


def _spans(mask, structure):
    lab, _ = ndimage.label(~mask.astype(bool), structure=structure)
    a = set(np.unique(lab[..., 0])) - {0}
    b = set(np.unique(lab[..., -1])) - {0}
    return bool(a & b)


@pytest.mark.parametrize("nx,ny,phi", _paper_2d())
def test_paper_resolutions_exact_porosity(nx, ny, phi):
    m = qsgs.qsgs_2d(nx, ny, phi, 0)
    assert m.shape == (ny, nx) and m.dtype == np.uint8
    assert int(m.sum()) == round((1 - phi) * nx * ny)
    assert _spans(m, np.ones((3, 3))) and qsgs.percolates(m)


def test_deterministic_and_seeded():
    a = qsgs.qsgs_2d(100, 50, 0.74, 3)
    b = qsgs.qsgs_2d(100, 50, 0.74, 3)
    c = qsgs.qsgs_2d(100, 50, 0.74, 4)
    assert (a == b).all() and (a != c).any()


def test_3d_exact_porosity_and_18_connected_percolation():
    m = qsgs.qsgs_3d(40, 32, 24, 0.6, 0)
    assert m.shape == (24, 32, 40)
    assert int(m.sum()) == round(0.4 * m.size)
    st = ndimage.generate_binary_structure(3, 2)  # faces + edges (D3Q19 links)
    assert _spans(m, st) and qsgs.percolates(m)


def test_clustered_growth():
    """Grown solids form blobs: far fewer solid clusters than solid cells."""
    m = qsgs.qsgs_2d(200, 100, 0.74, 1)
    _, n = ndimage.label(m.astype(bool), structure=np.ones((3, 3)))
    assert n < 0.05 * m.sum()


def test_percolation_detects_blocked_medium():
    m = np.zeros((10, 20), np.uint8)
    m[:, 7] = 1
    assert not qsgs.percolates(m)
    m[4, 7] = 0
    assert qsgs.percolates(m)


def test_invalid_arguments():
    with pytest.raises(qsgs.QSGSError):
        qsgs.qsgs_2d(0, 10, 0.7, 0)
    with pytest.raises(qsgs.QSGSError):
        qsgs.qsgs_2d(10, 10, 1.5, 0)


@pytest.mark.parametrize("shape,phi,seed", [((60, 90), 0.6, 3), ((40, 50), 0.75, 8),
                                            ((12, 20, 30), 0.6, 2)])
def test_open_fluid_matches_connected_components(shape, phi, seed):
    """Fluid connected to the inlet/outlet planes equals the union of the
    lattice-connected components (8 in 2D, 18 in 3D) touching x = 0 or nx-1."""
    import scipy.ndimage as ndi
    from paper_1609_09685_amd.qsgs import open_fluid, qsgs_2d, qsgs_3d
    if len(shape) == 2:
        m = qsgs_2d(shape[1], shape[0], phi, seed)
        st = np.ones((3, 3))
    else:
        m = qsgs_3d(shape[2], shape[1], shape[0], phi, seed)
        st = ndi.generate_binary_structure(3, 2)     # faces + edges
    lab, _ = ndi.label(m == 0, structure=st)
    ids = set(np.unique(lab[..., 0])) | set(np.unique(lab[..., -1]))
    ids.discard(0)
    ref = np.isin(lab, list(ids)).astype(np.uint8)
    got = open_fluid(m)
    assert np.array_equal(got, ref)
    # a closed pocket is excluded
    m2 = np.zeros((5, 8), np.uint8)
    m2[1:4, 3:6] = 1
    m2[2, 4] = 0
    o = open_fluid(m2)
    assert o[2, 4] == 0 and o[0, 0] == 1 and o.sum() == (m2 == 0).sum() - 1
