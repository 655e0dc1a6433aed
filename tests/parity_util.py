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
