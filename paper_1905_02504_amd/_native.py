"""Thin ctypes binding of the rg C-ABI (include/rg.h).

Argument marshalling only: every step of the method runs in the HIP library
(librg.so).  The functions keep the C names; device buffers and streams come
from PyTorch (tensor.data_ptr(), torch.cuda.current_stream().cuda_stream).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librg.so")

RG_OK, RG_EINVAL, RG_ENOMEM, RG_ESINGULAR, RG_ENOTSUP, RG_EDEVICE = range(6)
RG_MODE_FP64, RG_MODE_FP32, RG_MODE_BF16 = 0, 1, 2


class rg_mesh_desc(C.Structure):
    _fields_ = [("n_ang", C.c_int32), ("n_rad", C.c_int32), ("r_in", C.c_double), ("r_out", C.c_double),
                ("radial", C.c_int32), ("map_order", C.c_int32), ("n_ghost", C.c_int32)]


class rg_mesh_info(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("n_ang", "n_rad", "n_ghost", "n_shells", "n_columns", "n_zones",
                                         "n_faces", "n_radial_faces", "n_edges", "n_radial_edges",
                                         "n_vertices", "n_angular_edges")]


class rg_step_params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("dt", C.c_double), ("cfl", C.c_double), ("bc_kind", C.c_int32),
                ("n_picard", C.c_int32), ("weno_eps", C.c_double), ("fallback", C.c_int32),
                ("flattener", C.c_double)]


class rg_diag_out(C.Structure):
    _fields_ = [("div_rel_max", C.c_double), ("sums", C.c_double * 8), ("rho_min", C.c_double),
                ("p_min", C.c_double)]


class rg_prism_info(C.Structure):
    _fields_ = [("n_zones", C.c_int64), ("n_tri", C.c_int64), ("n_nodes", C.c_int32), ("n_levels", C.c_int32),
                ("order", C.c_int32), ("level", C.c_int32), ("n_rad", C.c_int32), ("n_face_points", C.c_int32),
                ("n_edges", C.c_int64), ("n_faces", C.c_int64), ("n_divfree_in", C.c_int32),
                ("n_divfree_out", C.c_int32), ("n_vertices", C.c_int64)]


class RGError(RuntimeError):
    pass


_lib = None
_vp = C.c_void_p
_dp = C.POINTER(C.c_double)


def lib():
    """Load librg.so; fails loudly when the HIP extension has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RGError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
        L = C.CDLL(LIB_PATH)
        L.rg_last_error.restype = C.c_char_p
        L.rg_mesh_build.argtypes = [C.POINTER(rg_mesh_desc), C.POINTER(_vp)]
        L.rg_mesh_get_info.argtypes = [_vp, C.POINTER(rg_mesh_info)]
        L.rg_mesh_free.argtypes = [_vp]
        L.rg_mesh_free.restype = None
        L.rg_geom_precompute.argtypes = [_vp, C.c_int32, C.c_int32, _vp, C.POINTER(_vp)]
        L.rg_geom_precompute_host.argtypes = [_vp, C.c_int32, C.POINTER(_vp)]
        L.rg_geom_free.argtypes = [_vp]
        L.rg_geom_free.restype = None
        L.rg_geom_zone_data.argtypes = [_vp, _vp, _vp]
        L.rg_geom_face_data.argtypes = [_vp, _vp, _vp, _vp]
        L.rg_geom_edge_data.argtypes = [_vp, _vp, _vp]
        L.rg_geom_incidence.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.rg_step.argtypes = [_vp, C.POINTER(rg_step_params), _vp, _vp, _vp, _vp, _vp]
        L.rg_step_fluxes.argtypes = [_vp, _vp, _vp, _vp]
        L.rg_step_fallback_zones.argtypes = [_vp, _vp, _vp]
        L.rg_step_weno_order.argtypes = [_vp, _vp, _vp]
        L.rg_fma_probe.argtypes = [_vp, C.c_int64, C.c_int32, _vp]
        L.rg_mfma_probe.argtypes = [_vp, C.c_int64, C.c_int32, C.c_int32, _vp]
        L.rg_step_adjoint.argtypes = [_vp, C.POINTER(rg_step_params), _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.rg_stokes.argtypes = [_vp, _vp, _vp, _vp]
        L.rg_stokes_T.argtypes = [_vp, _vp, _vp, _vp]
        L.rg_status_str.argtypes = [C.c_int]
        L.rg_status_str.restype = C.c_char_p
        L.rg_cfl_dt.argtypes = [_vp, _vp, C.c_double, C.c_double, _vp, _dp]
        L.rg_cfl_dt_noalloc.argtypes = [_vp, _vp, C.c_double, C.c_double, _vp, _dp]
        L.rg_geom_conditioning.argtypes = [_vp, _vp, _vp]
        L.rg_init_blast.argtypes = [_vp, _vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, _vp, _vp]
        L.rg_step_fallback_counts.argtypes = [_vp, _vp, _vp]
        L.rg_init_alfven.argtypes = [_vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_double, C.c_double, _vp, C.c_double, _vp, _vp]
        L.rg_init_tube.argtypes = [_vp, _vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                   _vp, _vp]
        L.rg_geom_work.argtypes = [_vp, _dp, _dp]
        L.rg_diag.argtypes = [_vp, _vp, _vp, C.c_double, _vp, C.POINTER(rg_diag_out)]
        L.rg_geom_work.restype = C.c_int
        L.rg_profile_begin.argtypes = [_vp]
        L.rg_profile_end.argtypes = [_vp, _dp, C.POINTER(C.c_int32)]
        L.rg_prism_build.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.POINTER(_vp)]
        L.rg_prism_build_host.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32, C.POINTER(_vp)]
        L.rg_prism_free.argtypes = [_vp]
        L.rg_prism_free.restype = None
        L.rg_prism_get_info.argtypes = [_vp, C.POINTER(rg_prism_info)]
        L.rg_prism_triangles.argtypes = [_vp, _vp]
        L.rg_prism_geometry.argtypes = [_vp, C.c_int64, C.c_int64, _vp, _vp, _vp]
        L.rg_prism_predict.argtypes = [_vp, C.c_double, C.c_double, C.c_int32, _vp, _vp, _vp, _vp]
        L.rg_prism_work.argtypes = [_vp, C.c_int32, _dp, _dp]
        L.rg_prism_face_points.argtypes = [_vp, _vp, _vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.rg_prism_traces.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.rg_prism_edges.argtypes = [_vp, _vp]
        L.rg_prism_face_fluxes.argtypes = [_vp, C.c_double, _vp, _vp, _vp]
        L.rg_prism_volumes.argtypes = [_vp, C.c_int64, C.c_int64, _vp]
        L.rg_prism_update.argtypes = [_vp, C.c_double, _vp, _vp, _vp, _vp]
        L.rg_prism_divfree.argtypes = [_vp, _vp, _vp, _vp]
        L.rg_prism_divfree_host.argtypes = [_vp, C.c_int64, C.c_int64, _vp, _vp]
        L.rg_prism_edge_traces.argtypes = [_vp, _vp, _vp, _vp, _vp]
        L.rg_prism_edge_emfs.argtypes = [_vp, C.c_double, _vp, _vp, _vp, _vp]
        L.rg_prism_ct.argtypes = [_vp, C.c_double, _vp, _vp, _vp, _vp, _vp]
        L.rg_prism_vertices.argtypes = [_vp, _vp]
        for name in ("rg_prism_build", "rg_prism_build_host", "rg_prism_get_info", "rg_prism_work",
                     "rg_prism_face_points", "rg_prism_traces", "rg_prism_edges", "rg_prism_face_fluxes",
                     "rg_prism_volumes", "rg_prism_update", "rg_prism_divfree", "rg_prism_divfree_host",
                     "rg_prism_edge_traces", "rg_prism_edge_emfs", "rg_prism_ct", "rg_prism_vertices", "rg_prism_triangles", "rg_prism_geometry",
                     "rg_prism_predict"):
            getattr(L, name).restype = C.c_int
        for name in ("rg_profile_begin", "rg_profile_end", "rg_mesh_build", "rg_mesh_get_info", "rg_geom_precompute", "rg_geom_precompute_host",
                     "rg_geom_zone_data", "rg_geom_face_data", "rg_geom_edge_data", "rg_geom_incidence", "rg_step",
                     "rg_step_fluxes",
                     "rg_step_fallback_zones", "rg_step_weno_order", "rg_fma_probe", "rg_mfma_probe",
                     "rg_step_adjoint", "rg_stokes", "rg_stokes_T", "rg_cfl_dt", "rg_init_alfven", "rg_init_tube", "rg_diag",
                     "rg_cfl_dt_noalloc", "rg_geom_conditioning", "rg_init_blast", "rg_step_fallback_counts"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != RG_OK:
        raise RGError(f"{what} failed ({lib().rg_status_str(status).decode()}): {lib().rg_last_error().decode()}")


# ------------------------------------------------------------------ C-ABI names
def rg_mesh_build(n_ang, n_rad, r_in=1.0, r_out=2.0, map_order=2, n_ghost=3):
    d = rg_mesh_desc(n_ang, n_rad, r_in, r_out, 0, map_order, n_ghost)
    h = _vp()
    check(lib().rg_mesh_build(C.byref(d), C.byref(h)), "rg_mesh_build")
    return h


def rg_mesh_get_info(mesh):
    info = rg_mesh_info()
    check(lib().rg_mesh_get_info(mesh, C.byref(info)), "rg_mesh_get_info")
    return {n: getattr(info, n) for n, _ in rg_mesh_info._fields_}


def rg_mesh_free(mesh):
    lib().rg_mesh_free(mesh)


def rg_geom_precompute(mesh, order, mode=RG_MODE_FP64, stream=0):
    h = _vp()
    check(lib().rg_geom_precompute(mesh, order, mode, _vp(stream), C.byref(h)), "rg_geom_precompute")
    return h


def rg_geom_precompute_host(mesh, order):
    h = _vp()
    check(lib().rg_geom_precompute_host(mesh, order, C.byref(h)), "rg_geom_precompute_host")
    return h


def rg_geom_free(geom):
    lib().rg_geom_free(geom)


def rg_geom_zone_data(geom, centroid_ptr, volume_ptr):
    check(lib().rg_geom_zone_data(geom, _vp(centroid_ptr), _vp(volume_ptr)), "rg_geom_zone_data")


def rg_geom_face_data(geom, center_ptr, normal_ptr, area_ptr):
    check(lib().rg_geom_face_data(geom, _vp(center_ptr), _vp(normal_ptr), _vp(area_ptr)), "rg_geom_face_data")


def rg_geom_edge_data(geom, mid_ptr, tan_ptr):
    check(lib().rg_geom_edge_data(geom, _vp(mid_ptr), _vp(tan_ptr)), "rg_geom_edge_data")


def rg_geom_incidence(geom, zf_ptr, zfs_ptr, fe_ptr, fes_ptr):
    check(lib().rg_geom_incidence(geom, _vp(zf_ptr), _vp(zfs_ptr), _vp(fe_ptr), _vp(fes_ptr)), "rg_geom_incidence")


def rg_step(geom, params: rg_step_params, U_ptr, Bf_ptr, Uo_ptr, Bfo_ptr, stream):
    check(lib().rg_step(geom, C.byref(params), _vp(U_ptr), _vp(Bf_ptr), _vp(Uo_ptr), _vp(Bfo_ptr), _vp(stream)),
          "rg_step")
    return params


def rg_step_adjoint(geom, params: rg_step_params, U_ptr, Bf_ptr, gU1_ptr, gBf1_ptr, gU_ptr, gBf_ptr, stream):
    check(lib().rg_step_adjoint(geom, C.byref(params), _vp(U_ptr), _vp(Bf_ptr), _vp(gU1_ptr), _vp(gBf1_ptr),
                                _vp(gU_ptr), _vp(gBf_ptr), _vp(stream)), "rg_step_adjoint")


def rg_stokes(geom, circ_ptr, Bf_ptr, stream):
    check(lib().rg_stokes(geom, _vp(circ_ptr), _vp(Bf_ptr), _vp(stream)), "rg_stokes")


def rg_stokes_T(geom, gBf_ptr, gcirc_ptr, stream):
    check(lib().rg_stokes_T(geom, _vp(gBf_ptr), _vp(gcirc_ptr), _vp(stream)), "rg_stokes_T")


def rg_status_str(status: int) -> str:
    return lib().rg_status_str(int(status)).decode()


def rg_step_fluxes(geom, Phi_ptr, Gam_ptr, stream):
    check(lib().rg_step_fluxes(geom, _vp(Phi_ptr), _vp(Gam_ptr), _vp(stream)), "rg_step_fluxes")


def rg_step_fallback_zones(geom, flags_ptr, stream):
    check(lib().rg_step_fallback_zones(geom, _vp(flags_ptr), _vp(stream)), "rg_step_fallback_zones")


def rg_step_weno_order(geom, whi_ptr, stream):
    check(lib().rg_step_weno_order(geom, _vp(whi_ptr), _vp(stream)), "rg_step_weno_order")


def rg_fma_probe(sink_ptr, n_threads, iters, stream):
    check(lib().rg_fma_probe(_vp(sink_ptr), int(n_threads), int(iters), _vp(stream)), "rg_fma_probe")


def rg_mfma_probe(sink_ptr, n_threads, iters, kind, stream):
    check(lib().rg_mfma_probe(_vp(sink_ptr), int(n_threads), int(iters), int(kind), _vp(stream)), "rg_mfma_probe")


def rg_cfl_dt(geom, U_ptr, gamma, cfl, stream):
    out = C.c_double(0.0)
    check(lib().rg_cfl_dt(geom, _vp(U_ptr), gamma, cfl, _vp(stream), C.byref(out)), "rg_cfl_dt")
    return out.value


def rg_cfl_dt_noalloc(geom, U_ptr, gamma, cfl, stream):
    out = C.c_double(0.0)
    check(lib().rg_cfl_dt_noalloc(geom, _vp(U_ptr), gamma, cfl, _vp(stream), C.byref(out)), "rg_cfl_dt_noalloc")
    return out.value


def rg_geom_conditioning(geom, lsq_ptr, kkt_ptr):
    check(lib().rg_geom_conditioning(geom, _vp(lsq_ptr), _vp(kkt_ptr)), "rg_geom_conditioning")


RG_FALLBACK_ROUNDS = 4


def rg_step_fallback_counts(geom, stream):
    out = (C.c_int32 * RG_FALLBACK_ROUNDS)()
    check(lib().rg_step_fallback_counts(geom, out, _vp(stream)), "rg_step_fallback_counts")
    return list(out)


def rg_init_blast(geom, axis_ptr, centre_ptr, radius, rho, p_in, p, B0, gamma, U_ptr, Bf_ptr):
    check(lib().rg_init_blast(geom, _vp(axis_ptr), _vp(centre_ptr), radius, rho, p_in, p, B0, gamma, _vp(U_ptr),
                              _vp(Bf_ptr)), "rg_init_blast")


def rg_init_tube(geom, left_ptr, right_ptr, Br0, r0, rm, delta, gamma, U_ptr, Bf_ptr):
    check(lib().rg_init_tube(geom, _vp(left_ptr), _vp(right_ptr), Br0, r0, rm, delta, gamma, _vp(U_ptr), _vp(Bf_ptr)),
          "rg_init_tube")


def rg_init_alfven(geom, frame_ptr, rho, p, B0, dB, wavelength, gamma, t, noise_ptr, noise_amp, U_ptr, Bf_ptr):
    check(lib().rg_init_alfven(geom, _vp(frame_ptr), rho, p, B0, dB, wavelength, gamma, t, _vp(noise_ptr),
                               noise_amp, _vp(U_ptr), _vp(Bf_ptr)), "rg_init_alfven")


def rg_diag(geom, U_ptr, Bf_ptr, gamma, stream):
    out = rg_diag_out()
    check(lib().rg_diag(geom, _vp(U_ptr), _vp(Bf_ptr), gamma, _vp(stream), C.byref(out)), "rg_diag")
    return {"div_rel_max": out.div_rel_max, "sums": list(out.sums), "rho_min": out.rho_min, "p_min": out.p_min}


STAGES = ("bc_fill", "weno", "face_bnodal", "bmap", "predictor", "face_flux", "edge_emf", "update_ct")
RG_NSTAGES = len(STAGES)


def rg_profile_begin(geom):
    check(lib().rg_profile_begin(geom), "rg_profile_begin")


def rg_profile_end(geom):
    ms = (C.c_double * RG_NSTAGES)()
    n = C.c_int32(0)
    check(lib().rg_profile_end(geom, ms, C.byref(n)), "rg_profile_end")
    return dict(zip(STAGES, list(ms))), n.value


def rg_geom_work(geom):
    f = (C.c_double * RG_NSTAGES)()
    b = (C.c_double * RG_NSTAGES)()
    check(lib().rg_geom_work(geom, f, b), "rg_geom_work")
    return dict(zip(STAGES, list(f))), dict(zip(STAGES, list(b)))


# ------------------------------------------------------------------ prism element
def rg_prism_build(level, n_rad, r_in, r_out, order):
    h = _vp()
    check(lib().rg_prism_build(level, n_rad, r_in, r_out, order, C.byref(h)), "rg_prism_build")
    return h


def rg_prism_build_host(level, n_rad, r_in, r_out, order):
    h = _vp()
    check(lib().rg_prism_build_host(level, n_rad, r_in, r_out, order, C.byref(h)), "rg_prism_build_host")
    return h


def rg_prism_free(prism):
    lib().rg_prism_free(prism)


def rg_prism_get_info(prism):
    info = rg_prism_info()
    check(lib().rg_prism_get_info(prism, C.byref(info)), "rg_prism_get_info")
    return {n: getattr(info, n) for n, _ in rg_prism_info._fields_}


def rg_prism_triangles(prism, abc_ptr):
    check(lib().rg_prism_triangles(prism, _vp(abc_ptr)), "rg_prism_triangles")


def rg_prism_geometry(prism, z0, nz, x_ptr, J_ptr, met_ptr):
    check(lib().rg_prism_geometry(prism, z0, nz, _vp(x_ptr), _vp(J_ptr), _vp(met_ptr)), "rg_prism_geometry")


def rg_prism_predict(prism, gamma, dt, n_picard, Ua_ptr, aU_ptr, aF_ptr, stream):
    check(lib().rg_prism_predict(prism, gamma, dt, n_picard, _vp(Ua_ptr), _vp(aU_ptr), _vp(aF_ptr), _vp(stream)),
          "rg_prism_predict")


def rg_prism_work(prism, n_picard):
    f, b = C.c_double(0), C.c_double(0)
    check(lib().rg_prism_work(prism, n_picard, C.byref(f), C.byref(b)), "rg_prism_work")
    return f.value, b.value


def rg_prism_face_points(prism, xi_ptr, w_ptr):
    nt, ns = C.c_int32(0), C.c_int32(0)
    check(lib().rg_prism_face_points(prism, _vp(xi_ptr), _vp(w_ptr), C.byref(nt), C.byref(ns)),
          "rg_prism_face_points")
    return nt.value, ns.value


def rg_prism_traces(prism, aU_ptr, aF_ptr, tr_ptr, stream):
    check(lib().rg_prism_traces(prism, _vp(aU_ptr), _vp(aF_ptr), _vp(tr_ptr), _vp(stream)), "rg_prism_traces")


def rg_prism_edges(prism, edges_ptr):
    check(lib().rg_prism_edges(prism, _vp(edges_ptr)), "rg_prism_edges")


def rg_prism_face_fluxes(prism, gamma, tr_ptr, Phi_ptr, stream):
    check(lib().rg_prism_face_fluxes(prism, gamma, _vp(tr_ptr), _vp(Phi_ptr), _vp(stream)), "rg_prism_face_fluxes")


def rg_prism_volumes(prism, z0, nz, vol_ptr):
    check(lib().rg_prism_volumes(prism, z0, nz, _vp(vol_ptr)), "rg_prism_volumes")


def rg_prism_update(prism, dt, U_ptr, Phi_ptr, Uo_ptr, stream):
    check(lib().rg_prism_update(prism, dt, _vp(U_ptr), _vp(Phi_ptr), _vp(Uo_ptr), _vp(stream)), "rg_prism_update")


def rg_prism_divfree(prism, Bin_ptr, Bout_ptr, stream):
    check(lib().rg_prism_divfree(prism, _vp(Bin_ptr), _vp(Bout_ptr), _vp(stream)), "rg_prism_divfree")


def rg_prism_divfree_host(prism, z0, nz, Bin_ptr, Bout_ptr):
    check(lib().rg_prism_divfree_host(prism, z0, nz, _vp(Bin_ptr), _vp(Bout_ptr)), "rg_prism_divfree_host")


def rg_prism_edge_traces(prism, aU_ptr, aF_ptr, er_ptr, stream):
    check(lib().rg_prism_edge_traces(prism, _vp(aU_ptr), _vp(aF_ptr), _vp(er_ptr), _vp(stream)), "rg_prism_edge_traces")


def rg_prism_edge_emfs(prism, gamma, er_ptr, Gang_ptr, Grad_ptr, stream):
    check(lib().rg_prism_edge_emfs(prism, gamma, _vp(er_ptr), _vp(Gang_ptr), _vp(Grad_ptr), _vp(stream)),
          "rg_prism_edge_emfs")


def rg_prism_ct(prism, dt, Gang_ptr, Grad_ptr, PhiB_ptr, PhiBo_ptr, stream):
    check(lib().rg_prism_ct(prism, dt, _vp(Gang_ptr), _vp(Grad_ptr), _vp(PhiB_ptr), _vp(PhiBo_ptr), _vp(stream)),
          "rg_prism_ct")


def rg_prism_vertices(prism, xyz_ptr):
    check(lib().rg_prism_vertices(prism, _vp(xyz_ptr)), "rg_prism_vertices")
