"""Host side of the library's prism element (no GPU): mesh and per-zone
geometry against the oracle's, counts and argument errors."""
import numpy as np
import pytest

from oracle import prism as P


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_geometry_matches_oracle(order):
    """Triangles (bit for bit: the same bisection), node positions, Jacobians
    and curl-form metrics of every zone of level 2 x 3 shells, each side
    computed from its own map (library: unit shell scaled per shell)."""
    import paper_1905_02504_amd as R
    lib = R.PrismMesh(2, 3, order, r_in=1.0, r_out=1.6, device=False)
    om = P.OraclePrismMesh(2, 3, r_in=1.0, r_out=1.6, order=order)
    assert (lib.nz, lib.ntri, lib.N) == (om.nz, om.ntri, om.N)
    assert np.array_equal(lib.triangles(), om.vert[om.tri])
    xo, Jo, mo = om.geometry(np.arange(om.nz))
    xl, Jl, ml = lib.geometry(0, lib.nz)
    assert np.abs(xl - xo).max() < 1e-14
    assert (np.abs(Jl - Jo) / np.abs(Jo)).max() < 1e-13
    assert np.abs(ml - mo).max() < 1e-12 * np.abs(mo).max()
    # a zone range in the middle
    x2, J2, m2 = lib.geometry(137, 5)
    assert np.array_equal(x2, xl[137:142]) and np.array_equal(m2, ml[137:142])


def test_prism_counts_and_errors():
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    for level in range(4):
        m = R.PrismMesh(level, 2, 3, device=False)
        assert m.ntri == 20 * 4 ** level and m.nz == 2 * m.ntri and m.N == 15
    for args in [(1, 2, 1.0, 2.0, 5), (9, 2, 1.0, 2.0, 4)]:
        with pytest.raises(N.RGError, match="RG_ENOTSUP"):
            N.rg_prism_build_host(*args)
    for args in [(1, 0, 1.0, 2.0, 4), (1, 2, 2.0, 1.0, 4), (1, 2, 0.0, 1.0, 4)]:
        with pytest.raises(N.RGError, match="RG_EINVAL"):
            N.rg_prism_build_host(*args)
    m = R.PrismMesh(0, 2, 4, device=False)
    with pytest.raises(N.RGError, match="host-only"):
        N.rg_prism_predict(m._h, 5 / 3, 0.01, 4, 8, 8, 8, 0)
    with pytest.raises(N.RGError, match="outside the mesh"):
        m.geometry(39, 2)


def test_prism_edges_and_face_counts_match_oracle():
    import paper_1905_02504_amd as R
    for level in (0, 1, 2):
        m = R.PrismMesh(level, 3, 3, device=False)
        om = P.OraclePrismMesh(level, 3, order=3)
        assert np.array_equal(m.edges(), om.edges())
        assert m.n_edges == 30 * 4 ** level and m.n_faces == m.ntri * 4 + m.n_edges * 3


def test_prism_volumes_match_oracle():
    import paper_1905_02504_amd as R
    for order in (2, 3, 4):
        m = R.PrismMesh(2, 3, order, r_in=1.0, r_out=1.5, device=False)
        om = P.OraclePrismMesh(2, 3, r_in=1.0, r_out=1.5, order=order)
        np.testing.assert_allclose(m.volumes(), om.volumes(np.arange(om.nz)), rtol=1e-13)


def permute_face_inputs(lib, order, Bin):
    """the oracle's inputs -> the library's: the face nodal part follows each
    side's own face-point order, matched by reference coordinates"""
    xl, _, _, _ = lib.face_points()
    xo, _, _, _ = P.face_points(order)
    j = np.linalg.norm(xl[:, None] - xo[None], axis=2).argmin(1)
    assert np.array_equal(np.sort(j), np.arange(len(xo)))
    f0 = 3 * (len(P.taylor_indices(order)) + 1)
    out = Bin.copy()
    out[:, f0:f0 + len(j)] = Bin[:, f0 + j]
    return out


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_divfree_map_matches_oracle(order):
    """The library's per-column divergence-free map (KKT solved for the unit
    shell, applied as a matrix) against the oracle's per-zone KKT solve on
    random inputs, every zone of level 1 x 3 shells (Section IV.b)."""
    import paper_1905_02504_amd as R
    lib = R.PrismMesh(1, 3, order, r_in=1.0, r_out=1.5, device=False)
    om = P.OraclePrismMesh(1, 3, r_in=1.0, r_out=1.5, order=order)
    assert (lib.n_divfree_in, lib.n_divfree_out) == P.divfree_sizes(order)
    Bin = np.random.default_rng(order).normal(size=(om.nz, lib.n_divfree_in))
    want = om.divfree(np.arange(om.nz), Bin)
    got = lib.divfree_host(permute_face_inputs(lib, order, Bin))
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # a zone range
    got2 = lib.divfree_host(permute_face_inputs(lib, order, Bin[100:107]), z0=100)
    assert np.array_equal(got2, got[100:107])
