"""Pins of the oracle's mesh and geometry (faces, area vectors, volumes,
centroids) against closed forms and integral identities.  The finite-volume
form of Sec. 2.1, Eq. (1) needs, per cell, its volume and outward face area
vectors; these tests fix them independently of the code that computes them."""
import numpy as np
import pytest

from paper_1704_01144_amd import inputs as I


@pytest.mark.parametrize("n,grading", [(2, 1.0), (5, 2.0), (12, 4.0)])
def test_face_counts_closed_form(orc, n, grading):
    nodes, tets = I.graded_cube_mesh(n, grading)
    m = orc.Mesh(nodes, tets)
    # 6 tets per hex; 12 triangles per hex interior + shared hex faces:
    # interior-of-hex faces 6 per hex, hex faces split in 2: 3*2 per hex plus
    # the boundary layer -> 12 n^3 + 6 n^2 faces, 12 n^2 of them on the boundary
    assert m.n_cells == 6 * n ** 3
    assert m.n_faces == 12 * n ** 3 + 6 * n ** 2
    assert m.n_boundary == 12 * n ** 2


@pytest.mark.parametrize("n,grading", [(3, 1.0), (12, 4.0), (16, 16.0)])
def test_volumes_and_integrals(orc, n, grading):
    nodes, tets = I.graded_cube_mesh(n, grading)
    m = orc.Mesh(nodes, tets)
    g = m.geometry()
    vol = g["vol"]
    assert (vol > 0).all()
    # the unit cube: total volume 1 and first moment 1/2 per axis
    assert abs(vol.sum() - 1.0) < 1e-13
    first = (vol[:, None] * g["centroid"]).sum(0)
    assert np.abs(first - 0.5).max() < 1e-13
    # the 6 tets of a hex fill it: volume = dx dy dz
    x = I.graded_coords(n, grading)
    d = np.diff(x)
    hexvol = (d[None, None, :] * d[None, :, None] * d[:, None, None]).ravel()  # k,j,i order
    assert np.abs(vol.reshape(-1, 6).sum(1) - hexvol).max() < 1e-15
    # the smallest and largest corner cells differ by the grading ratio cubed
    assert abs(vol.max() / vol.min() - grading ** 3) < 1e-9 * grading ** 3


def test_closure_and_divergence(orc):
    nodes, tets = I.graded_cube_mesh(6, 3.0)
    m = orc.Mesh(nodes, tets)
    g = m.geometry()
    L, R, A, xf, c2f = g["face_L"], g["face_R"], g["face_area"], g["face_centroid"], g["cell_faces"]
    cells = np.arange(m.n_cells)[:, None]
    sign = np.where(L[c2f] == cells, 1.0, -1.0)  # outward from each cell
    # closed surface: the outward area vectors of a cell sum to zero
    closure = (sign[..., None] * A[c2f]).sum(1)
    scale = np.abs(A).max()
    assert np.abs(closure).max() < 1e-14 * scale
    # divergence theorem for the field x: sum_f x_f . A_f = 3 V (exact for
    # planar faces with the centroid rule)
    flux_x = (sign * np.einsum("ijk,ijk->ij", xf[c2f], A[c2f])).sum(1)
    assert np.abs(flux_x - 3 * g["vol"]).max() < 1e-14
    # orientation: A points from L to R and out of the domain on the boundary
    inter = R >= 0
    dLR = g["centroid"][R[inter]] - g["centroid"][L[inter]]
    assert (np.einsum("ij,ij->i", A[inter], dLR) > 0).all()
    bnd = ~inter
    assert (np.einsum("ij,ij->i", A[bnd], xf[bnd] - 0.5) > 0).all()
    assert abs(np.linalg.norm(A[bnd], axis=1).sum() - 6.0) < 1e-13
    # every cell lists 4 distinct faces, interior faces have two distinct cells
    assert (np.sort(c2f, 1)[:, 1:] != np.sort(c2f, 1)[:, :-1]).all()
    assert (L[inter] < R[inter]).all()


def test_full_scale_mesh_counts(orc):
    # the 64^3 mesh with grading 16: 1,572,864 cells, 3,170,304 faces
    n = 64
    nodes, tets = I.graded_cube_mesh(n, 16.0)
    m = orc.Mesh(nodes, tets)
    assert (m.n_cells, m.n_faces, m.n_boundary) == (1572864, 3170304, 49152)
    vol = m.geometry()["vol"]
    assert abs(vol.sum() - 1.0) < 1e-12
    assert abs(vol.max() / vol.min() - 4096.0) < 1e-6


def test_malformed_meshes(orc):
    nodes, tets = I.graded_cube_mesh(2, 1.0)
    bad = tets.copy()
    bad[3, 2], bad[3, 3] = bad[3, 3], bad[3, 2]  # negative orientation
    with pytest.raises(orc.OracleError) as e:
        orc.Mesh(nodes, bad)
    assert e.value.code == orc.E_MESH
    bad = tets.copy()
    bad[0, 0] = len(nodes)  # vertex out of range
    with pytest.raises(orc.OracleError) as e:
        orc.Mesh(nodes, bad)
    assert e.value.code == orc.E_MESH
    # a face shared by three tets: duplicate a tet
    bad = np.concatenate([tets, tets[:1]])
    with pytest.raises(orc.OracleError) as e:
        orc.Mesh(nodes, bad)
    assert e.value.code == orc.E_MESH
