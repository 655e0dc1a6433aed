"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two small drivers are compiled with -fsanitize=address,undefined and run:
the oracle (one third- and one fourth-order step on tiny meshes), and the
library's host side (mesh build, geometry precompute without a device, the
host initialiser, argument errors, the prism element's mesh, geometry and
face points) with the device launchers replaced by stubs that refuse.  A sanitizer report makes the run exit non-zero.
"""
import os
import shutil
import subprocess
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_02504_amd", "csrc")
ODIR = os.path.join(ROOT, "oracle")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24", OMP_NUM_THREADS="2")

pytestmark = pytest.mark.slow

ORACLE_DRIVER = textwrap.dedent(r"""
    #include <stdint.h>
    #include <stdio.h>
    #include <stdlib.h>
    typedef struct rgo_mesh rgo_mesh;
    rgo_mesh *rgo_create(int, int, double, double, int, int, int);
    void rgo_destroy(rgo_mesh *);
    void rgo_sizes(const rgo_mesh *, int64_t *);
    int rgo_step(const rgo_mesh *, double, double, int, int, double, const double *, const double *, double *,
                 double *, double *, double *, unsigned char *);
    void rgo_init_tube(const rgo_mesh *, const double *, const double *, double, double, double, double, double,
                       double *, double *);
    static int run(int order, int ghost) {
        rgo_mesh *m = rgo_create(2, 3, 1.0, 2.0, ghost, order - 1, order);
        if (!m) return 1;
        int64_t s[8];
        rgo_sizes(m, s);
        int64_t nz = s[0], nf = s[1];
        double *U = calloc(8 * nz, sizeof(double)), *Bf = calloc(nf, sizeof(double));
        double *Uo = calloc(8 * nz, sizeof(double)), *Bo = calloc(nf, sizeof(double));
        for (int64_t z = 0; z < nz; z++) {
            double rho = 1.0 + 0.1 * ((z * 37) % 11) / 11.0, vx = 0.05 * ((z * 13) % 7) / 7.0;
            U[z] = rho; U[nz + z] = rho * vx; U[4 * nz + z] = 1.5 + 0.5 * rho * vx * vx;
        }
        /* a pressure hole that the high-order update drives negative: the
         * first-order fallback runs */
        U[4 * nz + nz / 2] = 1e-3 + 0.5 * U[nz + nz / 2] * U[nz + nz / 2] / U[nz / 2];
        unsigned char *fz = calloc(nz, 1);
        int rc = rgo_step(m, 5.0 / 3.0, 5e-2, 0, 2, 1e-4, U, Bf, Uo, Bo, NULL, NULL, fz);
        free(fz);
        for (int64_t i = 0; i < 8 * nz; i++) if (Uo[i] != Uo[i]) rc = 2;
        /* the spherical shock tube's initial state */
        const double tl[7] = {1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0}, tr[7] = {0.125, 0.1, 0.0, 0.0, 0.0, 0.0, -1.0};
        rgo_init_tube(m, tl, tr, 0.75, 1.5, 1.5, 0.01, 2.0, U, Bf);
        for (int64_t i = 0; i < 8 * nz; i++) if (U[i] != U[i]) rc = 3;
        free(U); free(Bf); free(Uo); free(Bo);
        rgo_destroy(m);
        return rc;
    }
    int main(void) {
        int rc = run(3, 2) | run(4, 3);
        printf("oracle driver rc=%d\n", rc);
        return rc;
    }
""")

LIB_DRIVER = textwrap.dedent(r"""
    #include <cstdio>
    #include <vector>
    #include "rg_geom_host.hpp"
    #include "prism.hpp"
    namespace rg {
    // the device side is not linked: every launcher refuses
    rg_status launch_step(rg_geom *, const rg_step_params &, const double *, const double *, double *, double *, void *) { return RG_ENOTSUP; }
    rg_status profile_end(rg_geom *, double *, int *) { return RG_ENOTSUP; }
    rg_status launch_cfl(rg_geom *, const double *, double, double, void *, double *) { return RG_ENOTSUP; }
    rg_status launch_cfl_noalloc(rg_geom *, const double *, double, double, void *, double *) { return RG_ENOTSUP; }
    rg_status launch_step_front(rg_geom *, const rg_step_params &, const double *, const double *, double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_adjoint(rg_geom *, const rg_step_params &, const double *, const double *, const double *, const double *, double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_stokes(rg_geom *, const double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_stokes_T(rg_geom *, const double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_diag(rg_geom *, const double *, const double *, double, void *, rg_diag_out *) { return RG_ENOTSUP; }
    rg_status launch_fma_probe(double *, long long, int, void *) { return RG_ENOTSUP; }
    rg_status launch_mfma_probe(double *, long long, int, int, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_predict(const DevPrism &, double, double, int, const double *, double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_traces(const DevPrism &, const double *, const double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_face_flux(const DevPrism &, double, const double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_update(const DevPrism &, double, const double *, const double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_divfree(const DevPrism &, const double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_edge_traces(const DevPrism &, const double *, const double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_edge_emfs(const DevPrism &, double, const double *, double *, double *, void *) { return RG_ENOTSUP; }
    rg_status launch_prism_ct(const DevPrism &, double, const double *, const double *, const double *, double *, void *) { return RG_ENOTSUP; }
    }
    // the prism element's host side: mesh, geometry and face-point queries
    static int run_prism(int order) {
        rg_prism *p = nullptr;
        if (rg_prism_build_host(2, 3, 1.0, 1.6, order, &p) != RG_OK) { std::printf("%s\n", rg_last_error()); return 10; }
        rg_prism_info info;
        rg_prism_get_info(p, &info);
        std::vector<double> abc(9 * info.n_tri), x(3 * 5 * info.n_nodes), J(5 * info.n_nodes), met(45 * info.n_nodes);
        std::vector<double> xi(3 * info.n_face_points), w(info.n_face_points);
        int rc = rg_prism_triangles(p, abc.data());
        if (rc == RG_OK) rc = rg_prism_geometry(p, info.n_zones - 5, 5, x.data(), J.data(), met.data());
        int32_t nt = 0, ns = 0;
        if (rc == RG_OK) rc = rg_prism_face_points(p, xi.data(), w.data(), &nt, &ns);
        double f = 0, b = 0;
        if (rc == RG_OK) rc = rg_prism_work(p, order, &f, &b);
        std::vector<int32_t> edges(4 * info.n_edges);
        if (rc == RG_OK) rc = rg_prism_edges(p, edges.data());
        if (rg_prism_face_fluxes(p, 5.0 / 3.0, x.data(), x.data(), nullptr) != RG_EINVAL) rc = 14;
        std::vector<double> vol(info.n_zones);
        if (rc == RG_OK) rc = rg_prism_volumes(p, 0, info.n_zones, vol.data());
        if (rg_prism_update(p, 1e-3, x.data(), x.data(), x.data(), nullptr) != RG_EINVAL) rc = 15;
        std::vector<double> bin(3 * info.n_divfree_in, 0.5), bout(3 * info.n_divfree_out);
        if (rc == RG_OK) rc = rg_prism_divfree_host(p, info.n_zones - 3, 3, bin.data(), bout.data());
        if (rg_prism_divfree_host(p, info.n_zones - 2, 3, bin.data(), bout.data()) != RG_EINVAL) rc = 16;
        if (rg_prism_divfree(p, bin.data(), bout.data(), nullptr) != RG_EINVAL) rc = 17;
        std::vector<double> vxyz(3 * info.n_vertices);
        if (rc == RG_OK) rc = rg_prism_vertices(p, vxyz.data());
        if (rg_prism_edge_traces(p, x.data(), x.data(), x.data(), nullptr) != RG_EINVAL) rc = 18;
        if (rg_prism_edge_emfs(p, 5.0 / 3.0, x.data(), x.data(), x.data(), nullptr) != RG_EINVAL) rc = 20;
        if (rg_prism_ct(p, 1e-3, x.data(), x.data(), x.data(), x.data(), nullptr) != RG_EINVAL) rc = 19;
        if (rg_prism_geometry(p, info.n_zones - 4, 5, x.data(), J.data(), met.data()) != RG_EINVAL) rc = 11;
        if (rg_prism_predict(p, 5.0 / 3.0, 1e-3, order, x.data(), x.data(), x.data(), nullptr) != RG_EINVAL) rc = 12;
        rg_prism_free(p);
        if (rg_prism_build_host(9, 3, 1.0, 1.6, order, &p) != RG_ENOTSUP) rc = 13;
        return rc;
    }
    static int run(int order) {
        rg_mesh_desc d{4, 3, 1.0, 2.0, 0, order - 1, 3};
        rg_mesh *m = nullptr;
        if (rg_mesh_build(&d, &m) != RG_OK) return 1;
        rg_mesh_info info;
        rg_mesh_get_info(m, &info);
        rg_geom *g = nullptr;
        if (rg_geom_precompute_host(m, order, &g) != RG_OK) { std::printf("%s\n", rg_last_error()); return 2; }
        std::vector<double> cen(3 * info.n_zones), vol(info.n_zones), U(8 * info.n_zones), Bf(info.n_faces);
        std::vector<double> fc(3 * info.n_faces), fn(3 * info.n_faces), fa(info.n_faces);
        std::vector<double> em(3 * info.n_edges), et(3 * info.n_edges);
        rg_geom_zone_data(g, cen.data(), vol.data());
        rg_geom_face_data(g, fc.data(), fn.data(), fa.data());
        rg_geom_edge_data(g, em.data(), et.data());
        const double frame[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        int rc = rg_init_alfven(g, frame, 1.0, 0.1, 1.0, 0.1, 1.0, 5.0 / 3.0, 0.0, nullptr, 0.0, U.data(), Bf.data());
        const double tl[7] = {1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0}, tr[7] = {0.125, 0.1, 0.0, 0.0, 0.0, 0.0, -1.0};
        if (rc == RG_OK) rc = rg_init_tube(g, tl, tr, 0.75, 1.5, 1.5, 0.01, 2.0, U.data(), Bf.data());
        const double tbad[7] = {1.0, 1.0, 0.0, 0.0, 0.0, 0.5, 1.0};
        if (rc == RG_OK && rg_init_tube(g, tbad, tr, 0.75, 1.5, 1.5, 0.01, 2.0, U.data(), Bf.data()) != RG_EINVAL) rc = 4;
        const double axis[3] = {0.0, 0.0, 1.0}, centre[3] = {0.0, 0.0, 1.5};
        if (rc == RG_OK)
            rc = rg_init_blast(g, axis, centre, 0.3, 1.0, 1000.0, 0.1, 1.0, 5.0 / 3.0, U.data(), Bf.data());
        std::vector<double> cl(info.n_columns), ck(info.n_columns);
        if (rc == RG_OK) rc = rg_geom_conditioning(g, cl.data(), ck.data());
        std::vector<int64_t> zf(6 * info.n_zones), fe(4 * info.n_faces);
        std::vector<int8_t> zs(6 * info.n_zones), fs(4 * info.n_faces);
        if (rc == RG_OK) rc = rg_geom_incidence(g, zf.data(), zs.data(), fe.data(), fs.data());
        // without device data the step entry points refuse
        rg_step_params p{5.0 / 3.0, 1e-3, 0.0, 0, 0, 0.0};
        if (rg_step(g, &p, U.data(), Bf.data(), U.data(), Bf.data(), nullptr) == RG_OK) rc = 3;
        double work_f[RG_NSTAGES], work_b[RG_NSTAGES];
        rg_geom_work(g, work_f, work_b);
        rg_geom_free(g);
        rg_mesh_free(m);
        return rc;
    }
    int main() {
        rg_mesh *m = nullptr;
        rg_mesh_desc bad{10, 3, 1.0, 2.0, 0, 2, 3};   // neither 2^k nor 3 x 2^k
        int rc = rg_mesh_build(&bad, &m) == RG_OK;
        rc |= run(3) | run(4);
        rc |= run_prism(2) | run_prism(3) | run_prism(4);
        std::printf("library host driver rc=%d\n", rc);
        return rc;
    }
""")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    drv = tmp_path / "oracle_driver.c"
    drv.write_text(ORACLE_DRIVER)
    from oracle import oracle as O
    srcs = [os.path.join(ODIR, s) for s in O._SOURCES]
    exe = tmp_path / "oracle_driver"
    subprocess.run(["gcc", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", *SAN, str(drv), *srcs, "-o", str(exe), "-lm"],
                   check=True, capture_output=True)
    res = subprocess.run([str(exe)], env=ENV, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]


def test_library_host_side_under_sanitizers(tmp_path):
    _need("g++")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.exists(os.path.join(rocm, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("HIP headers not available")
    drv = tmp_path / "lib_driver.cpp"
    drv.write_text(LIB_DRIVER)
    srcs = [os.path.join(CSRC, s) for s in ("mesh.cpp", "refel.cpp", "geom.cpp", "init.cpp", "capi.cpp",
                                            "prism_ref.cpp", "prism.cpp")]
    exe = tmp_path / "lib_driver"
    cmd = ["g++", "-std=c++17", "-fopenmp", *SAN, "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", str(drv), *srcs, "-o", str(exe),
           f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=0:exitcode=23")   # the HIP runtime's own allocations
    res = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]
