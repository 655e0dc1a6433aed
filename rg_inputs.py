"""Seeded synthetic inputs shared by the oracle and the GPU library.

This module holds no arithmetic of the numerical method.  It only turns seeds
into problem-definition parameters:

* scalar fields on the sphere, sum_{l<=4, m} c_lm Y_lm(x/|x|) with real
  orthonormal spherical harmonics (no Condon-Shortley phase, (l, m) in
  lexicographic order, m = -l..l) and coefficients c_lm ~ N(0, 1) / (l+1)^2,
  re-expressed as homogeneous polynomials: f(x) = sum_k a_k x^e_k / |x|^deg_k
  over the 35 monomials of degree <= 4 listed by MONOMIALS;
* the propagation axis and transverse frame of a circularly polarised wave;
* the parameters of a magnetised blast and its piecewise-constant pressure;
* the spherical Sod shock tube (a radial jump in density and pressure);
* per-zone white-noise arrays.

The two consumers (the oracle under oracle/ and the library's field
initialiser) each evaluate these definitions with their own code.
"""
from __future__ import annotations

import math

import numpy as np

LMAX = 4

# monomials x^a y^b z^c of degree <= 4: by degree, then a descending, b descending
MONOMIALS = [(a, b, d - a - b) for d in range(LMAX + 1)
             for a in range(d, -1, -1) for b in range(d - a, -1, -1)]
N_MONO = len(MONOMIALS)  # 35

SEED_RHO = 101
SEED_V = (102, 103, 104)
SEED_A = (105, 106, 107)
SEED_AXIS = 108
SEED_NOISE = 109
SEED_TARGET = (110, 111)


def _assoc_legendre(l: int, m: int, x: np.ndarray) -> np.ndarray:
    """P_l^m(x) without the Condon-Shortley phase, m >= 0."""
    pmm = np.ones_like(x)
    if m > 0:
        s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
        fact = 1.0
        for _ in range(m):
            pmm = pmm * fact * s
            fact += 2.0
    if l == m:
        return pmm
    pmmp1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pmmp1
    pll = pmmp1
    for ll in range(m + 2, l + 1):
        pll = (x * (2 * ll - 1) * pmmp1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pmmp1 = pmmp1, pll
    return pll


def real_ylm(l: int, m: int, n: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonic at unit vectors n (..., 3)."""
    ct = n[..., 2]
    phi = np.arctan2(n[..., 1], n[..., 0])
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi)
                     * math.factorial(l - am) / math.factorial(l + am))
    p = _assoc_legendre(l, am, ct)
    if m == 0:
        return norm * p
    if m > 0:
        return math.sqrt(2.0) * norm * p * np.cos(am * phi)
    return math.sqrt(2.0) * norm * p * np.sin(am * phi)


def _ylm_as_monomials() -> dict:
    """Exact homogeneous-polynomial form of each Y_lm (degree l)."""
    rng = np.random.default_rng(12345)
    pts = rng.normal(size=(200, 3))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    out = {}
    for l in range(LMAX + 1):
        idx = [k for k, e in enumerate(MONOMIALS) if sum(e) == l]
        V = np.stack([pts[:, 0] ** MONOMIALS[k][0] * pts[:, 1] ** MONOMIALS[k][1]
                      * pts[:, 2] ** MONOMIALS[k][2] for k in idx], axis=1)
        for m in range(-l, l + 1):
            y = real_ylm(l, m, pts)
            c, *_ = np.linalg.lstsq(V, y, rcond=None)
            if np.max(np.abs(V @ c - y)) > 1e-12:
                raise RuntimeError("Y_lm is not a homogeneous polynomial fit")
            full = np.zeros(N_MONO)
            full[idx] = c
            out[(l, m)] = full
    return out


_YLM_MONO = None


def harmonic_field(seed: int) -> np.ndarray:
    """Monomial coefficients (35,) of sum_lm c_lm Y_lm, c_lm ~ N(0,1)/(l+1)^2."""
    global _YLM_MONO
    if _YLM_MONO is None:
        _YLM_MONO = _ylm_as_monomials()
    rng = np.random.default_rng(seed)
    out = np.zeros(N_MONO)
    for l in range(LMAX + 1):
        for m in range(-l, l + 1):
            out += rng.normal() / (l + 1) ** 2 * _YLM_MONO[(l, m)]
    return out


def eval_field(coef: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Evaluate a field given by monomial coefficients at points x (..., 3)."""
    r = np.linalg.norm(x, axis=-1)
    val = np.zeros(x.shape[:-1])
    for k, (a, b, c) in enumerate(MONOMIALS):
        val = val + coef[k] * x[..., 0] ** a * x[..., 1] ** b * x[..., 2] ** c / r ** (a + b + c)
    return val


def harmonic_problem() -> dict:
    """Smooth multi-harmonic state: rho = 1 + 0.1 f, p = 1, v = 0.1 f, A = 0.1 f.

    Returns monomial-coefficient arrays of shape (35,) for rho (including the
    constant 1), vx, vy, vz and the vector potential Ax, Ay, Az.
    """
    rho = 0.1 * harmonic_field(SEED_RHO)
    rho[0] += 1.0
    return {
        "rho": rho,
        "v": np.stack([0.1 * harmonic_field(s) for s in SEED_V]),
        "A": np.stack([0.1 * harmonic_field(s) for s in SEED_A]),
        "p": 1.0,
        "gamma": 5.0 / 3.0,
    }


def wave_frame(seed: int = SEED_AXIS) -> np.ndarray:
    """Seeded unit axis a and transverse e1, e2 with e1 x e2 = a; rows (e1, e2, a)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    helper = np.eye(3)[int(np.argmin(np.abs(a)))]
    e1 = np.cross(a, helper)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(a, e1)
    return np.stack([e1, e2, a])


def alfven_problem() -> dict:
    """Circularly polarised Alfven wave: B0 = 1 along a, dB = 0.1, rho = 1, p = 0.1."""
    return {"frame": wave_frame(), "rho": 1.0, "p": 0.1, "B0": 1.0, "dB": 0.1,
            "wavelength": 1.0, "gamma": 5.0 / 3.0}


def blast_problem(p_in: float = 1000.0, radius: float = 0.1) -> dict:
    """Magnetised blast, after the blast problem of Section VIII.b rescaled to the
    shell 1 <= r <= 2: rho = 1, v = 0, p = 0.1, gamma = 1.4, uniform B of
    magnitude 10 / sqrt(4 pi) along the seeded axis a (plasma beta 2p/B^2 about
    0.025, rationalised units), and p = p_in inside the ball of the given
    radius centred at 1.5 a."""
    frame = wave_frame()
    return {"frame": frame, "rho": 1.0, "p": 0.1, "B0": 10.0 / math.sqrt(4.0 * math.pi), "dB": 0.0,
            "wavelength": 1.0, "gamma": 1.4, "p_in": p_in, "radius": radius, "centre": 1.5 * frame[2],
            "axis": frame[2].copy()}


def blast_pressure(prob: dict, centroids: np.ndarray) -> np.ndarray:
    """Per-zone pressure of the blast: p_in for zones whose centroid lies in the ball, p elsewhere."""
    inside = np.linalg.norm(centroids - prob["centre"], axis=1) < prob["radius"]
    return np.where(inside, prob["p_in"], prob["p"])


def sod_problem() -> dict:
    """Spherical Sod shock tube (Section VIII.c): shell 2 <= r <= 3, (rho, p, v) =
    (1, 1, 0) for r <= 2.5 and (0.125, 0.1, 0) outside, B = 0, gamma = 1.4,
    final time 0.2."""
    return {"r_in": 2.0, "r_out": 3.0, "r0": 2.5, "left": (1.0, 0.0, 1.0), "right": (0.125, 0.0, 0.1),
            "gamma": 1.4, "t_end": 0.2}


def sod_primitives(prob: dict, centroids: np.ndarray) -> tuple:
    """Per-zone (rho, p) of the Sod problem from each zone's centroid radius."""
    inner = np.linalg.norm(centroids, axis=1) <= prob["r0"]
    rho = np.where(inner, prob["left"][0], prob["right"][0])
    p = np.where(inner, prob["left"][2], prob["right"][2])
    return rho, p


SQRT4PI = float(np.sqrt(4.0 * np.pi))


def _tube(r_in, r_out, n_rad, left, right, Br0, gamma, t_end):
    rm = 4.5
    return {"r_in": r_in, "r_out": r_out, "left": tuple(left), "right": tuple(right), "Br0": Br0, "r0": 4.5,
            "rm": rm, "delta": 0.5 * rm * np.log(r_out / r_in) / n_rad, "gamma": gamma, "t_end": t_end}


def brio_wu_problem(n_rad: int) -> dict:
    """Spherical Brio-Wu tube (Section VIII.c), pole on the z axis: shell
    4 <= r <= 6, states (rho, p, v_r, v_theta, v_phi, B_theta, B_phi) =
    (1, 1, 0, 0, 0, 0, 1) for r <= 4.5 and (0.125, 0.1, 0, 0, 0, 0, -1) outside,
    B_r = 0.75 sin(theta) (4.5 / r)^2, gamma = 2, final time 0.1.  The paper
    gives the fields in units with magnetic pressure B^2 / (8 pi); here they are
    divided by sqrt(4 pi) for the step's B^2 / 2.  The toroidal field's taper
    is half the zone width at r = 4.5 for n_rad geometric shells."""
    return _tube(4.0, 6.0, n_rad, (1.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0), (0.125, 0.1, 0.0, 0.0, 0.0, 0.0, -1.0),
                 0.75, 2.0, 0.1)


def ryu_jones_problem(n_rad: int) -> dict:
    """Spherical Ryu-Jones tube (Section VIII.c): shell 3 <= r <= 6, states
    (1, 20, 10, 0, 0, 0, 5) for r <= 4.5 and (1, 1, -10, 0, 0, 0, 5) outside,
    B_r = 5 sin(theta) (4.5 / r)^2, gamma = 5/3, final time 0.06; fields
    divided by sqrt(4 pi) as for brio_wu_problem."""
    b = 5.0 / SQRT4PI
    return _tube(3.0, 6.0, n_rad, (1.0, 20.0, 10.0, 0.0, 0.0, 0.0, b), (1.0, 1.0, -10.0, 0.0, 0.0, 0.0, b),
                 b, 5.0 / 3.0, 0.06)


def white_noise(n: int, seed: int = SEED_NOISE, count: int = 2) -> np.ndarray:
    """Uniform(-1, 1) noise, shape (count, n)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(count, n))


def loss_targets(n: int, rho0: float = 1.0, b0: float = 1.0, amp: float = 0.01) -> tuple:
    """Per-zone targets (rho*, b*) of the adjoint checks' loss:
    rho0 (1 + amp U(-1,1)) from SEED_TARGET[0] and b0 (1 + amp U(-1,1)) from SEED_TARGET[1]."""
    r = np.random.default_rng(SEED_TARGET[0]).uniform(-1.0, 1.0, size=n)
    b = np.random.default_rng(SEED_TARGET[1]).uniform(-1.0, 1.0, size=n)
    return rho0 * (1.0 + amp * r), b0 * (1.0 + amp * b)
