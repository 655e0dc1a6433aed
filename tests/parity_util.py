"""Helpers shared by the parity tests: build both sides, map the oracle's
zone/face/edge numbering onto the library's by matching coordinates, and the
per-zone relative error measure."""
import numpy as np
from scipy.spatial import cKDTree


def match(points_lib, points_ref, tol=1e-9):
    d, idx = cKDTree(points_ref).query(points_lib)
    assert d.max() < tol * max(1.0, np.abs(points_ref).max()), f"unmatched points (max distance {d.max()})"
    assert len(np.unique(idx)) == len(idx), "matching is not one-to-one"
    return idx


class Mapping:
    """Index maps library <- oracle for zones, faces (with orientation) and edges."""

    def __init__(self, lib_shell, omesh):
        pc, _ = lib_shell.zone_data()
        oc, _, _, _ = omesh.zones()
        self.z = match(pc, oc)
        pfc, pfn, _ = lib_shell.face_data()
        ofc, ofn, _, _ = omesh.faces()
        self.f = match(pfc, ofc)
        self.fs = np.sign(np.einsum("ij,ij->i", pfn, ofn[self.f]))
        pem, pet = lib_shell.edge_data()
        oem, oet, _ = omesh.edges()
        self.e = match(pem, oem)
        self.es = np.sign(np.einsum("ij,ij->i", pet, oet[self.e]))

    def U(self, U_oracle):
        return np.ascontiguousarray(U_oracle[:, self.z])

    def Bf(self, Bf_oracle):
        return np.ascontiguousarray(self.fs * Bf_oracle[self.f])

    def Phi(self, Phi_oracle):  # oracle (nf, 8) -> library (8, nf)
        return np.ascontiguousarray((self.fs[:, None] * Phi_oracle[self.f]).T)

    def Gam(self, Gam_oracle):
        return np.ascontiguousarray(self.es * Gam_oracle[self.e])


def rel_err(x, ref):
    """Per-entry |x - ref| / max(|ref|, rms of ref over the same variable)."""
    x = np.atleast_2d(x); ref = np.atleast_2d(ref)
    rms = np.sqrt(np.mean(ref * ref, axis=1, keepdims=True))
    scale = np.maximum(np.abs(ref), rms)
    scale = np.where(scale == 0, 1.0, scale)
    return np.abs(x - ref) / scale


def roughen(U_h, Bf_h, gam, amp=0.2, seed=4242):
    """per-zone noise of relative size amp in rho, p and of size amp in v and B
    (primitive variables; total energy rebuilt), and amp x rms noise in face B"""
    rng = np.random.default_rng(seed)
    U = U_h.copy()
    rho = U[0]
    v = U[1:4] / rho
    B = U[5:8]
    p = (gam - 1) * (U[4] - 0.5 * rho * (v * v).sum(0) - 0.5 * (B * B).sum(0))
    rho = rho * (1 + amp * rng.uniform(-1, 1, rho.shape))
    p = p * (1 + amp * rng.uniform(-1, 1, p.shape))
    v = v + amp * rng.uniform(-1, 1, v.shape)
    B = B + amp * rng.uniform(-1, 1, B.shape)
    U[0] = rho
    U[1:4] = rho * v
    U[5:8] = B
    U[4] = p / (gam - 1) + 0.5 * rho * (v * v).sum(0) + 0.5 * (B * B).sum(0)
    Bf = Bf_h + amp * np.sqrt((Bf_h ** 2).mean()) * rng.uniform(-1, 1, Bf_h.shape)
    return U, Bf
