"""Parity of the library's prism-element kernels (predictor, face traces, face
fluxes, update and the divergence-free reconstruction of B) with the
oracle's on the same inputs, zone by zone:
small icosahedral meshes at orders 2-4 (every zone, ragged last workgroups),
the fourth-order benchmark mesh (level 6, 128 shells) on sampled zones, a
uniform state at full size, and the argument errors."""
import numpy as np
import pytest

from oracle import prism as P

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0
TOL = 1e-12


def smooth_state(x, rng, noise=0.01):
    """conserved MHD state [.., 8] from a smooth field at positions x plus
    seeded multiplicative noise"""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    rho = 1.0 + 0.2 * np.sin(3 * X) * np.sin(2 * Y + Z)
    v = np.stack([0.3 * np.sin(Y), 0.3 * np.cos(Z), 0.3 * np.sin(X)], -1)
    p = 1.0 + 0.1 * np.cos(X + Y)
    B = np.stack([0.4 + 0.1 * np.sin(Z), 0.2 * np.cos(X), 0.3 * np.sin(Y)], -1)
    rho = rho * (1 + noise * rng.uniform(-1, 1, rho.shape))
    p = p * (1 + noise * rng.uniform(-1, 1, p.shape))
    U = np.empty(x.shape[:-1] + (8,))
    U[..., 0] = rho
    U[..., 1:4] = rho[..., None] * v
    U[..., 4] = p / (GAMMA - 1) + 0.5 * rho * (v * v).sum(-1) + 0.5 * (B * B).sum(-1)
    U[..., 5:8] = B
    return U


def rel_by_var(a, b, axis):
    """max |a - b| / max |b| for each variable (variables on `axis`); a
    variable that vanishes identically (the flux of B_d along d) is measured
    against the largest variable's scale"""
    a = np.moveaxis(a, axis, 0).reshape(a.shape[axis], -1)
    b = np.moveaxis(b, axis, 0).reshape(b.shape[axis], -1)
    scale = np.abs(b).max(1)
    return np.abs(a - b).max(1) / np.maximum(scale, 1e-3 * scale.max())


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("level,n_rad,dt", [(0, 5, 0.05), (1, 3, 0.02)])
def test_prism_predictor_matches_oracle(order, level, n_rad, dt):
    import paper_1905_02504_amd as R
    print(f"[prism] order {order}, level {level} x {n_rad} shells, dt {dt}", flush=True)
    lib = R.PrismMesh(level, n_rad, order, r_in=1.0, r_out=1.5)
    om = P.OraclePrismMesh(level, n_rad, r_in=1.0, r_out=1.5, order=order)
    zones = np.arange(om.nz)
    x, J, met = om.geometry(zones)
    Ua = smooth_state(x, np.random.default_rng(100 * order + level))
    aU_o, aF_o = P.predict(order, J, met, Ua, dt, GAMMA)
    Ua_d = torch.from_numpy(np.ascontiguousarray(Ua.transpose(2, 0, 1))).cuda()
    aU, aF = lib.predict(Ua_d, dt, GAMMA)
    torch.cuda.synchronize()
    eU = rel_by_var(aU.cpu().numpy(), aU_o.transpose(2, 0, 1), 0)
    eF = rel_by_var(aF.cpu().numpy().reshape(24, om.nz, om.N), aF_o.reshape(om.nz, om.N, 24).transpose(2, 0, 1), 0)
    print(f"[prism] max rel error per variable: avgU {eU.max():.2e}, avgF {eF.max():.2e}", flush=True)
    assert eU.max() < TOL and eF.max() < TOL


def _point_map(lib, order):
    """library face point q -> the oracle's point at the same coordinates"""
    xl, wl, nt, ns = lib.face_points()
    xo, wo, nto, nso = P.face_points(order)
    assert (nt, ns) == (nto, nso)
    d = np.linalg.norm(xl[:, None, :] - xo[None, :, :], axis=2)
    j = d.argmin(1)
    assert d.min(1).max() < 1e-14 and len(set(j.tolist())) == len(j)
    np.testing.assert_allclose(wl, wo[j], rtol=0, atol=1e-15)
    return j


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_traces_match_oracle(order):
    """Face-point traces (rg_prism_traces) of the library's averages against the
    oracle's traces of its own averages, level 1 x 3 shells (ragged last
    workgroup at every order)."""
    import paper_1905_02504_amd as R
    print(f"[prism] traces, order {order}, level 1 x 3 shells", flush=True)
    lib = R.PrismMesh(1, 3, order, r_in=1.0, r_out=1.5)
    om = P.OraclePrismMesh(1, 3, r_in=1.0, r_out=1.5, order=order)
    x, J, met = om.geometry(np.arange(om.nz))
    Ua = smooth_state(x, np.random.default_rng(7 + order))
    aU_o, aF_o = P.predict(order, J, met, Ua, 0.02, GAMMA)
    tr_o = P.traces(order, aU_o, aF_o)                           # [z][q][32]
    aU, aF = lib.predict(torch.from_numpy(np.ascontiguousarray(Ua.transpose(2, 0, 1))).cuda(), 0.02, GAMMA)
    tr = lib.traces(aU, aF).cpu().numpy().transpose(0, 2, 1)     # [32][q][z] -> [32][z][q]
    j = _point_map(lib, order)
    e = rel_by_var(tr, tr_o[:, j, :].transpose(2, 0, 1), 0)
    print(f"[prism] traces: max rel error per value {e.max():.2e}", flush=True)
    assert e.max() < TOL


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_face_fluxes_match_oracle(order):
    """HLL face-flux integrals (rg_prism_face_fluxes) over every radial and
    side face of level 1 x 3 shells, from the library's own predictor and
    traces, against the oracle's chain on the same inputs."""
    import paper_1905_02504_amd as R
    print(f"[prism] face fluxes, order {order}, level 1 x 3 shells", flush=True)
    lib = R.PrismMesh(1, 3, order, r_in=1.0, r_out=1.5)
    om = P.OraclePrismMesh(1, 3, r_in=1.0, r_out=1.5, order=order)
    x, J, met = om.geometry(np.arange(om.nz))
    Ua = smooth_state(x, np.random.default_rng(31 + order))
    aU_o, aF_o = P.predict(order, J, met, Ua, 0.02, GAMMA)
    Phi_o = om.face_fluxes(P.traces(order, aU_o, aF_o), GAMMA)
    aU, aF = lib.predict(torch.from_numpy(np.ascontiguousarray(Ua.transpose(2, 0, 1))).cuda(), 0.02, GAMMA)
    Phi = lib.face_fluxes(lib.traces(aU, aF), GAMMA).cpu().numpy()
    assert Phi.shape == Phi_o.shape == (lib.n_faces, 8)
    e = rel_by_var(Phi, Phi_o, 1)
    print(f"[prism] face fluxes ({lib.n_faces} faces): max rel error per variable {e.max():.2e}", flush=True)
    assert e.max() < TOL


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_update_matches_oracle(order):
    """The finite-volume update (rg_prism_update) of zone averages from the
    library's own face fluxes against the oracle's chain, level 1 x 3."""
    import paper_1905_02504_amd as R
    print(f"[prism] update, order {order}, level 1 x 3 shells", flush=True)
    lib = R.PrismMesh(1, 3, order, r_in=1.0, r_out=1.5)
    om = P.OraclePrismMesh(1, 3, r_in=1.0, r_out=1.5, order=order)
    x, J, met = om.geometry(np.arange(om.nz))
    Ua = smooth_state(x, np.random.default_rng(53 + order))
    U = Ua.mean(1)                                  # zone averages [nz][8]
    dt = 0.02
    aU_o, aF_o = P.predict(order, J, met, Ua, dt, GAMMA)
    U1_o = om.update(U, om.face_fluxes(P.traces(order, aU_o, aF_o), GAMMA), dt)
    aU, aF = lib.predict(torch.from_numpy(np.ascontiguousarray(Ua.transpose(2, 0, 1))).cuda(), dt, GAMMA)
    Phi = lib.face_fluxes(lib.traces(aU, aF), GAMMA)
    U1 = lib.update(torch.from_numpy(np.ascontiguousarray(U.T)).cuda(), Phi, dt).cpu().numpy()
    e = rel_by_var(U1, U1_o.T, 0)
    print(f"[prism] update: max rel error per variable {e.max():.2e}", flush=True)
    assert e.max() < TOL


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_predictor_converges_at_design_order(order):
    """A density advected by uniform v with uniform p and B is an exact ideal-MHD
    solution.  From its nodal values at t^n the predictor's time-averaged
    density at every node of the curved prisms approaches the exact time
    average at the design order p as the icosahedral level and the shell count
    are refined together (dt halving with the zones; Section VII's claim for
    the scheme)."""
    import paper_1905_02504_amd as R
    print(f"[prism] convergence, order {order}", flush=True)
    v = np.array([0.3, -0.2, 0.1]); B = np.array([0.1, 0.2, 0.3]); p = 1.0
    rho0 = lambda x: 1.0 + 0.2 * np.sin(2 * x[..., 0]) * np.cos(x[..., 1]) * np.sin(x[..., 2] + 0.3)
    gt, gw = np.polynomial.legendre.leggauss(8)
    gt, gw = 0.5 * (gt + 1), 0.5 * gw
    errs = []
    for L in (2, 3, 4):
        lib = R.PrismMesh(L, 2 ** L, order, r_in=1.0, r_out=1.5)
        x, _, _ = lib.geometry(0, lib.nz)
        dt = 0.1 / 2 ** L
        r = rho0(x)
        U = np.zeros((8,) + r.shape)
        U[0] = r
        U[1:4] = r[None] * v[:, None, None]
        U[4] = p / (GAMMA - 1) + 0.5 * r * (v @ v) + 0.5 * (B @ B)
        U[5:8] = B[:, None, None]
        aU, _ = lib.predict(torch.from_numpy(np.ascontiguousarray(U)).cuda(), dt, GAMMA)
        exact = sum(w * rho0(x - v * t * dt) for t, w in zip(gt, gw))
        errs.append(float(np.abs(aU[0].cpu().numpy() - exact).max()))
        lib.close()
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(f"[prism] order {order}: max error {errs}, rates {np.round(rates, 2)}", flush=True)
    assert min(rates) > order - 0.5, (errs, rates)


def test_prism_predictor_without_sweeps_returns_the_initial_state():
    """n_picard = 0 keeps every level at the initial state: the averages are
    the state itself and its physical flux (the Gauss weights sum to one)."""
    import paper_1905_02504_amd as R
    from oracle import oracle as O
    print("[prism] n_picard = 0, order 4, level 0 x 2", flush=True)
    lib = R.PrismMesh(0, 2, 4)
    om = P.OraclePrismMesh(0, 2, order=4)
    x, _, _ = om.geometry(np.arange(om.nz))
    Ua = smooth_state(x, np.random.default_rng(3))
    aU, aF = lib.predict(torch.from_numpy(np.ascontiguousarray(Ua.transpose(2, 0, 1))).cuda(), 0.05, GAMMA,
                         n_picard=0)
    aU = aU.cpu().numpy().transpose(1, 2, 0)
    aF = aF.cpu().numpy().transpose(2, 3, 0, 1)
    np.testing.assert_allclose(aU, Ua, rtol=1e-14, atol=0)
    F = np.array([[O.flux(u) for u in zu] for zu in Ua])
    np.testing.assert_allclose(aF, F, rtol=0, atol=1e-13 * np.abs(F).max())


def _to_lib_inputs(lib, order, Bin):
    """oracle KKT inputs [z][nin] -> the library's [nin][z] (the face nodal
    part in the library's face-point order)"""
    j = _point_map(lib, order)
    f0 = 3 * (len(P.taylor_indices(order)) + 1)
    out = Bin.copy()
    out[:, f0:f0 + len(j)] = Bin[:, f0 + j]
    return np.ascontiguousarray(out.T)


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("level,n_rad,cols", [(1, 3, None), (0, 70, [0, 7, 19])])
def test_prism_divfree_matches_oracle(order, level, n_rad, cols):
    """The divergence-free reconstruction of B (rg_prism_divfree, Section
    IV.b on five faces) against the oracle's per-zone KKT solve on seeded
    random inputs: every zone of level 1 x 3 shells (3 of 64 lanes live), and
    every shell of three columns of level 0 x 70 (a full and a ragged run of
    64 shells)."""
    import paper_1905_02504_amd as R
    print(f"[prism] divfree, order {order}, level {level} x {n_rad} shells", flush=True)
    lib = R.PrismMesh(level, n_rad, order, r_in=1.0, r_out=1.5)
    om = P.OraclePrismMesh(level, n_rad, r_in=1.0, r_out=1.5, order=order)
    Bin = np.random.default_rng(71 + order).normal(size=(lib.nz, lib.n_divfree_in))
    out = lib.divfree(torch.from_numpy(_to_lib_inputs(lib, order, Bin)).cuda()).cpu().numpy()
    zones = np.arange(lib.nz) if cols is None else np.concatenate([np.arange(c * n_rad, (c + 1) * n_rad) for c in cols])
    want = om.divfree(zones, Bin[zones])
    e = np.abs(out[:, zones].T - want).max() / np.abs(want).max()
    print(f"[prism] divfree: {len(zones)} zones, max error {e:.2e} of the largest output", flush=True)
    assert e < TOL


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_divfree_reproduces_linear_divergence_free_field(order):
    """Inputs of a trace-free linear field B0 + G x (div B = 0, in the space
    at every order) come back exactly at the nodes of every zone of level
    1 x 3 shells, with the zone means at the centroids."""
    import paper_1905_02504_amd as R
    from tests.test_oracle_prism import divfree_inputs_linear
    lib = R.PrismMesh(1, 3, order, r_in=1.0, r_out=1.5)
    om = P.OraclePrismMesh(1, 3, r_in=1.0, r_out=1.5, order=order)
    rng = np.random.default_rng(5)
    G = rng.normal(size=(3, 3)); G -= np.eye(3) * np.trace(G) / 3
    B0 = rng.normal(size=3)
    zones = np.arange(lib.nz)
    Bin = divfree_inputs_linear(om, zones, B0, G)
    out = lib.divfree(torch.from_numpy(_to_lib_inputs(lib, order, Bin)).cuda()).cpu().numpy().T
    x, _, _ = lib.geometry(0, lib.nz)
    N = lib.N
    got = out[:, :3 * N].reshape(lib.nz, 3, N).transpose(0, 2, 1)
    np.testing.assert_allclose(got, B0[None, None] + x @ G.T, rtol=0, atol=1e-12)
    cen, _ = om.frames(zones)
    np.testing.assert_allclose(out[:, 3 * N:], B0[None] + cen @ G.T, rtol=0, atol=1e-12)


def _fullsize():
    import paper_1905_02504_amd as R
    return R.PrismMesh(6, 128, 4, r_in=1.0, r_out=2.0)


@pytest.fixture
def release_device_memory():
    """The full-size arrays take about 190 GB; hand them back to the device
    (not only to torch's cache) so that later tests can allocate."""
    yield
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_prism_predictor_fullsize_sampled_zones(release_device_memory):
    """The benchmark's launch: order 4 on level 6 (81,920 triangles) x 128
    shells, 10.5 M zones; uniform state with 5 % seeded noise; sampled zones
    (first, last, spread in between) against the oracle."""
    print("[prism] full size: order 4, level 6 x 128 shells, sampled zones", flush=True)
    lib = _fullsize()
    gen = torch.Generator(device="cuda").manual_seed(7)
    base = torch.tensor([1.0, 0.3, -0.2, 0.1, 2.0, 0.4, 0.2, -0.3], dtype=torch.float64, device="cuda")
    Ua = base[:, None, None] * (1 + 0.05 * (2 * torch.rand((8, lib.nz, lib.N), generator=gen, device="cuda",
                                                             dtype=torch.float64) - 1))
    dt = 2e-3
    aU, aF = lib.predict(Ua, dt, GAMMA)
    torch.cuda.synchronize()
    assert torch.isfinite(aU).all() and torch.isfinite(aF).all()
    om = P.OraclePrismMesh(6, 128, r_in=1.0, r_out=2.0, order=4)
    zones = np.unique(np.concatenate([[0, 1, 127, 128, lib.nz - 1, lib.nz - 2],
                                      np.random.default_rng(9).integers(0, lib.nz, 18)]))
    zt = torch.from_numpy(zones).cuda()
    Us = Ua[:, zt].cpu().numpy().transpose(1, 2, 0)
    _, J, met = om.geometry(zones)
    aU_o, aF_o = P.predict(4, J, met, np.ascontiguousarray(Us), dt, GAMMA)
    eU = rel_by_var(aU[:, zt].cpu().numpy(), aU_o.transpose(2, 0, 1), 0)
    eF = rel_by_var(aF[:, :, zt].cpu().numpy().reshape(24, len(zones), 26),
                    aF_o.reshape(len(zones), 26, 24).transpose(2, 0, 1), 0)
    print(f"[prism] {len(zones)} sampled zones: avgU {eU.max():.2e}, avgF {eF.max():.2e}", flush=True)
    assert eU.max() < TOL and eF.max() < TOL
    # face traces of the whole mesh, sampled zones against the oracle's
    tr = lib.traces(aU, aF)
    tr_o = P.traces(4, aU_o, aF_o)
    j = _point_map(lib, 4)
    eT = rel_by_var(tr[:, :, zt].cpu().numpy().transpose(0, 2, 1), tr_o[:, j, :].transpose(2, 0, 1), 0)
    print(f"[prism] sampled traces: {eT.max():.2e}", flush=True)
    assert eT.max() < TOL
    # face fluxes and the update of the whole mesh: conservation up to the
    # boundary fluxes, zone averages from the nodal states
    Phi = lib.face_fluxes(tr, GAMMA)
    del tr
    U = Ua.mean(2).contiguous()
    U1 = lib.update(U, Phi, dt)
    vol = torch.from_numpy(lib.volumes()).cuda()
    nr = lib.n_rad
    rad = torch.arange(lib.ntri, device="cuda") * (nr + 1)
    outer, inner = Phi[rad + nr].sum(0), Phi[rad].sum(0)
    lhs = (vol[None, :] * (U1 - U)).sum(1)
    rhs = -dt * (outer - inner)
    scale = float(dt * (Phi.abs() * 1.0).sum(0).max())
    dev_c = float((lhs - rhs).abs().max()) / scale
    print(f"[prism] update at full size: conservation defect {dev_c:.2e} of the summed face fluxes", flush=True)
    assert dev_c < 1e-12 and torch.isfinite(U1).all()
    del Phi, U, U1
    # free stream at full size: a uniform state stays uniform in every zone
    Ua.copy_(base[:, None, None].expand_as(Ua))
    aU, aF = lib.predict(Ua, dt, GAMMA, aU=aU, aF=aF)
    dev = float((aU - Ua).abs().max() / base.abs().max())
    print(f"[prism] uniform state: max relative change {dev:.2e}", flush=True)
    del Ua, aU, aF, base
    lib.close()
    assert dev < 1e-12


def test_prism_divfree_fullsize_sampled_zones(release_device_memory):
    """The benchmark's launch of rg_prism_divfree: order 4, level 6 x 128
    shells (10.5 M zones, 5.5 GB of column maps), seeded random inputs,
    sampled zones against the oracle."""
    print("[prism] full size divfree: order 4, level 6 x 128 shells, sampled zones", flush=True)
    lib = _fullsize()
    gen = torch.Generator(device="cuda").manual_seed(11)
    Bin = torch.randn((lib.n_divfree_in, lib.nz), generator=gen, device="cuda", dtype=torch.float64)
    out = lib.divfree(Bin)
    torch.cuda.synchronize()
    om = P.OraclePrismMesh(6, 128, r_in=1.0, r_out=2.0, order=4)
    zones = np.unique(np.concatenate([[0, 63, 64, 127, 128, lib.nz - 1],
                                      np.random.default_rng(13).integers(0, lib.nz, 18)]))
    zt = torch.from_numpy(zones).cuda()
    Bl = Bin[:, zt].cpu().numpy()                    # library order [nin][z]
    j = _point_map(lib, 4)
    f0 = 3 * (len(P.taylor_indices(4)) + 1)
    Bo = Bl.T.copy()
    Bo[:, f0 + j] = Bl.T[:, f0:f0 + len(j)]          # back to the oracle's face-point order
    want = om.divfree(zones, Bo)
    e = np.abs(out[:, zt].cpu().numpy().T - want).max() / np.abs(want).max()
    print(f"[prism] full size divfree: {len(zones)} sampled zones, max error {e:.2e}", flush=True)
    del Bin, out
    lib.close()
    assert e < TOL


def test_prism_predictor_argument_errors():
    import paper_1905_02504_amd as R
    from paper_1905_02504_amd import _native as N
    print("[prism] argument errors", flush=True)
    lib = R.PrismMesh(0, 1, 3)
    U = torch.zeros((8, lib.nz, lib.N), dtype=torch.float64, device="cuda")
    for g, dt, npic in [(1.0, 0.1, 3), (5 / 3, -1.0, 3), (5 / 3, 0.1, -1), (5 / 3, 0.1, 17)]:
        with pytest.raises(N.RGError, match="RG_EINVAL"):
            N.rg_prism_predict(lib._h, g, dt, npic, U.data_ptr(), U.data_ptr(), U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_predict(lib._h, 5 / 3, 0.1, 3, 0, U.data_ptr(), U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_traces(lib._h, U.data_ptr(), 0, U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_face_fluxes(lib._h, 1.0, U.data_ptr(), U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_update(lib._h, -1.0, U.data_ptr(), U.data_ptr(), U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_divfree(lib._h, 0, U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_edge_traces(lib._h, U.data_ptr(), 0, U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_edge_emfs(lib._h, 1.0, U.data_ptr(), U.data_ptr(), U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_edge_emfs(lib._h, 5 / 3, U.data_ptr(), 0, U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_ct(lib._h, -1.0, U.data_ptr(), U.data_ptr(), U.data_ptr(), U.data_ptr(), 0)
    with pytest.raises(N.RGError, match="RG_EINVAL"):
        N.rg_prism_ct(lib._h, 0.1, U.data_ptr(), U.data_ptr(), 0, U.data_ptr(), 0)


def _vertex_map(lib, om):
    """library vertex i -> the oracle's vertex at the same coordinates"""
    V = lib.vertices()
    d = np.linalg.norm(V[:, None, :] - om.vert[None, :, :], axis=2)
    j = d.argmin(1)
    assert d.min(1).max() == 0.0 and len(set(j.tolist())) == len(j)
    return j


@pytest.mark.parametrize("order", [2, 3, 4])
def test_prism_edge_emfs_and_ct_match_oracle(order):
    """Edge integrals of E (rg_prism_edge_emfs: four-state field at angular
    edges, two-zone field at r_in and r_out, the K-face mean at the five- and
    six-zone radial edges) from the library's predictor, and the face flux
    update (rg_prism_ct), against the oracle's chain on the same nodal
    states, level 1 x 3 shells; every zone's net outward flux kept."""
    import paper_1905_02504_amd as R
    print(f"[prism] edge fields and CT, order {order}, level 1 x 3 shells", flush=True)
    lib = R.PrismMesh(1, 3, order, r_in=1.0, r_out=1.5)
    om = P.OraclePrismMesh(1, 3, r_in=1.0, r_out=1.5, order=order)
    x, J, met = om.geometry(np.arange(om.nz))
    Ua = smooth_state(x, np.random.default_rng(91 + order))
    dt = 0.02
    aU_o, aF_o = P.predict(order, J, met, Ua, dt, GAMMA)
    Ga_o, Gr_o = om.edge_emfs(aU_o, aF_o, GAMMA)
    aU, aF = lib.predict(torch.from_numpy(np.ascontiguousarray(Ua.transpose(2, 0, 1))).cuda(), dt, GAMMA)
    Ga, Gr = lib.edge_emfs(lib.edge_traces(aU, aF), GAMMA)
    Ga, Gr = Ga.cpu().numpy(), Gr.cpu().numpy()
    vm = _vertex_map(lib, om)
    scale = max(np.abs(Ga_o).max(), np.abs(Gr_o).max())
    ea, er = np.abs(Ga - Ga_o).max() / scale, np.abs(Gr - Gr_o[vm]).max() / scale
    print(f"[prism] edge integrals: angular {ea:.2e}, radial {er:.2e} of the largest", flush=True)
    assert ea < TOL and er < TOL
    # constrained transport from random face fluxes
    nf = lib.n_faces
    Phi0 = np.random.default_rng(5).normal(size=nf)
    want = om.ct_update(Phi0, Ga_o, Gr_o, dt)
    got = lib.ct(torch.from_numpy(Phi0).cuda(), torch.from_numpy(Ga).cuda(), torch.from_numpy(Gr).cuda(), dt)
    got = got.cpu().numpy()
    ect = np.abs(got - want).max() / np.abs(want).max()
    # the change alone (from zero fluxes): each zone's net outward flux stays zero
    d = lib.ct(torch.zeros(nf, dtype=torch.float64, device="cuda"), torch.from_numpy(Ga).cuda(),
               torch.from_numpy(Gr).cuda(), dt).cpu().numpy()
    F, S = om.zone_faces()
    div = np.abs((S * d[F]).sum(1)).max() / np.abs(d).max()
    print(f"[prism] CT: {ect:.2e} of the largest flux; zone net flux change {div:.2e} of the largest change",
          flush=True)
    assert ect < TOL and div < 1e-14


def test_prism_ct_fullsize_keeps_zone_fluxes(release_device_memory):
    """The benchmark mesh (order 4, level 6 x 128 shells): edge integrals
    from the predictor of a noisy state and one CT update from zero face
    fluxes; every zone's net outward flux stays zero to round-off, and a
    uniform state changes no face flux."""
    print("[prism] full size edge fields and CT", flush=True)
    lib = _fullsize()
    gen = torch.Generator(device="cuda").manual_seed(21)
    base = torch.tensor([1.0, 0.3, -0.2, 0.1, 2.0, 0.4, 0.2, -0.3], dtype=torch.float64, device="cuda")
    Ua = base[:, None, None] * (1 + 0.05 * (2 * torch.rand((8, lib.nz, lib.N), generator=gen, device="cuda",
                                                             dtype=torch.float64) - 1))
    dt = 2e-3
    aU, aF = lib.predict(Ua, dt, GAMMA)
    er = lib.edge_traces(aU, aF)
    Ga, Gr = lib.edge_emfs(er, GAMMA)
    zero = torch.zeros(lib.n_faces, dtype=torch.float64, device="cuda")
    dPhi = lib.ct(zero, Ga, Gr, dt)
    torch.cuda.synchronize()
    assert torch.isfinite(Ga).all() and torch.isfinite(Gr).all()
    nr, nt = lib.n_rad, lib.ntri
    nrf = nt * (nr + 1)
    t = torch.arange(nt, device="cuda")[:, None] * (nr + 1) + torch.arange(nr, device="cuda")[None, :]
    net = (dPhi[t + 1] - dPhi[t]).reshape(-1)           # zone t nr + k: top minus bottom
    E = torch.from_numpy(lib.edges().astype(np.int64)).cuda()
    ks = torch.arange(nr, device="cuda")
    side = dPhi[nrf:].reshape(-1, nr)
    net.index_add_(0, (E[:, 0:1] * nr + ks[None, :]).reshape(-1), side.reshape(-1))
    net.index_add_(0, (E[:, 2:3] * nr + ks[None, :]).reshape(-1), -side.reshape(-1))
    rel = float(net.abs().max() / dPhi.abs().max())
    print(f"[prism] full size CT: zone net flux change {rel:.2e} of the largest face change", flush=True)
    assert rel < 1e-13
    Ua.copy_(base[:, None, None].expand_as(Ua))
    aU, aF = lib.predict(Ua, dt, GAMMA, aU=aU, aF=aF)
    Ga, Gr = lib.edge_emfs(lib.edge_traces(aU, aF, er), GAMMA, Ga, Gr)
    dPhi2 = lib.ct(zero, Ga, Gr, dt)
    uni = float(dPhi2.abs().max() / dPhi.abs().max())
    print(f"[prism] full size CT, uniform state: largest face change {uni:.2e} of the noisy one", flush=True)
    del Ua, aU, aF, er, Ga, Gr, dPhi, dPhi2, zero, net, side
    lib.close()
    assert uni < 1e-9
