"""FP64 CPU oracle for the SPECT OSEM hot path of the paper.

TEST INFRASTRUCTURE ONLY.  The checker for the HIP library: only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` import
this module.  It shares no code with the product path (the HIP library and its
binding); the only module both sides use is the seeded input generator
``paper_2309_01977_amd.phantoms``, which holds none of the method's arithmetic.

Contents
  * ``forward`` / ``back``: the system matrix H of Eq. 1 (Section 2.1.1) and
    its transpose, computed in FP64 by ``spect_oracle.c`` (plain loops).
  * ``poisson_gradient``: the Poisson log-likelihood gradient of Table 1,
    H^T (g / (H f + s)) - H^T 1.
  * ``osem``: the preconditioned gradient ascent update of Eq. 5 with the OSEM
    preconditioner of Table 1, f / (H^(n)T 1), and no prior (V = 0), over
    M subsets of the projection angles (Section 2.1.3).
  * ``dense_matrix``: H as an explicit matrix for tiny grids (brute force).
  * ``rdp_value`` / ``rdp_gradient`` / ``bsrem``: the relative difference
    prior of Table 1 and BSREM (Eq. 4 with the Table 1 preconditioner).
  * ``unrolled_osem_grad``: the mean-squared error of K unrolled OSEM
    subiterations to a target image and its gradient with respect to the
    initial image, by the chain rule applied to the update backwards (the
    reference for the differentiable projector pair).

Readings where the paper is silent (also listed in the C source):
  subsets are interleaved (angle n belongs to subset n mod M) and are visited
  in order m = 0..M-1; the initial image is 1 everywhere; the data ratio is 0
  where the expected projection is not positive; a voxel with zero subset
  sensitivity keeps its value.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spect_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libspect_oracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        os.makedirs(os.path.dirname(_LIB), exist_ok=True)
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("nz", ctypes.c_int), ("n_angles", ctypes.c_int),
                ("voxel_cm", ctypes.c_double), ("psf_a", ctypes.c_double),
                ("psf_b", ctypes.c_double), ("psf_nsigma", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_forward.argtypes = [ctypes.POINTER(_Geom), dp, dp, dp, dp, ip, ctypes.c_int, dp]
        lib.orc_forward.restype = ctypes.c_int
        lib.orc_back.argtypes = [ctypes.POINTER(_Geom), dp, dp, dp, dp, ip, ctypes.c_int, dp]
        lib.orc_back.restype = ctypes.c_int
        lib.orc_psf_taps.argtypes = [ctypes.POINTER(_Geom), ctypes.c_double, ctypes.c_int, dp,
                                     ctypes.c_int]
        lib.orc_psf_taps.restype = ctypes.c_int
        lib.orc_trig.argtypes = [ctypes.c_double, dp, dp]
        lib.orc_rotate.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_double, dp]
        lib.orc_rotate_adjoint.argtypes = lib.orc_rotate.argtypes
        _lib = lib
    return _lib


@dataclass
class Geometry:
    """Parallel-hole SPECT acquisition on an N x N x Nz grid of cubic voxels.

    angles_deg: gantry angles (default n * 360 / A); radius_cm: distance from
    the rotation axis to the detector face per angle (default N * dx / 2);
    psf_a, psf_b: collimator-detector sigma(d) = a d + b in cm (0, 0 = none);
    psf_nsigma: truncation radius in sigmas.
    """
    n: int
    nz: int
    n_angles: int
    voxel_cm: float
    psf_a: float = 0.0
    psf_b: float = 0.0
    psf_nsigma: float = 4.0
    angles_deg: Optional[Sequence[float]] = None
    radius_cm: Optional[Sequence[float]] = None

    def _c(self):
        g = _Geom(self.n, self.nz, self.n_angles, self.voxel_cm, self.psf_a, self.psf_b,
                  self.psf_nsigma)
        ang = None if self.angles_deg is None else np.ascontiguousarray(self.angles_deg, np.float64)
        rad = None if self.radius_cm is None else np.ascontiguousarray(self.radius_cm, np.float64)
        return g, ang, rad

    @property
    def object_shape(self):
        return (self.n, self.n, self.nz)

    @property
    def proj_shape(self):
        return (self.n_angles, self.n, self.nz)


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _idx(geom: Geometry, idx):
    if idx is None:
        idx = np.arange(geom.n_angles)
    return np.ascontiguousarray(idx, dtype=np.int32)


def forward(geom: Geometry, f, mu=None, idx=None, out=None) -> np.ndarray:
    """Rows idx of H f (Eq. 1); other rows of ``out`` are left as they are.
    The rows are a set: an angle listed twice is projected once (its row is
    not summed twice, and two threads never write one row)."""
    lib = _load()
    g, ang, rad = geom._c()
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(geom.object_shape)
    mu = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64).reshape(geom.object_shape)
    ix = np.ascontiguousarray(np.unique(_idx(geom, idx)), dtype=np.int32)
    if out is None:
        out = np.zeros(geom.proj_shape, dtype=np.float64)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape == geom.proj_shape
    st = lib.orc_forward(ctypes.byref(g), _dp(ang), _dp(rad), _dp(f), _dp(mu),
                         ix.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(ix), _dp(out))
    if st != 0:
        raise ValueError("oracle forward: blur radius beyond the oracle's limit")
    return out


def back(geom: Geometry, proj, mu=None, idx=None) -> np.ndarray:
    """sum over n in idx of H_n^T proj[n] (transpose of Eq. 1)."""
    lib = _load()
    g, ang, rad = geom._c()
    proj = np.ascontiguousarray(proj, dtype=np.float64).reshape(geom.proj_shape)
    mu = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64).reshape(geom.object_shape)
    ix = _idx(geom, idx)
    out = np.zeros(geom.object_shape, dtype=np.float64)
    st = lib.orc_back(ctypes.byref(g), _dp(ang), _dp(rad), _dp(proj), _dp(mu),
                      ix.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(ix), _dp(out))
    if st != 0:
        raise ValueError("oracle back: blur radius beyond the oracle's limit")
    return out


def psf_taps(geom: Geometry, depth: int, angle: int = 0) -> np.ndarray:
    """One-sided collimator-detector taps g[0..K] at rotated depth ``depth``."""
    lib = _load()
    g, _, rad = geom._c()
    R = 0.5 * geom.n * geom.voxel_cm if rad is None else float(rad[angle])
    buf = np.zeros(257, dtype=np.float64)
    K = lib.orc_psf_taps(ctypes.byref(g), R, int(depth), _dp(buf), 256)
    if K < 0:
        raise ValueError("blur radius beyond the oracle's limit")
    return buf[:K + 1].copy()


def trig(deg: float):
    lib = _load()
    c, s = ctypes.c_double(), ctypes.c_double()
    lib.orc_trig(float(deg), ctypes.byref(c), ctypes.byref(s))
    return c.value, s.value


def rotate(vol, deg: float) -> np.ndarray:
    """T_rot alone: the bilinear rotated volume [i'][j'][k]."""
    lib = _load()
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    N, _, Nz = vol.shape
    c, s = trig(deg)
    out = np.zeros_like(vol)
    lib.orc_rotate(_dp(vol), N, Nz, c, s, _dp(out))
    return out


def rotate_adjoint(rot, deg: float) -> np.ndarray:
    lib = _load()
    rot = np.ascontiguousarray(rot, dtype=np.float64)
    N, _, Nz = rot.shape
    c, s = trig(deg)
    out = np.zeros_like(rot)
    lib.orc_rotate_adjoint(_dp(rot), N, Nz, c, s, _dp(out))
    return out


def subsets(n_angles: int, n_subsets: int):
    """Interleaved partition of the angles: subset m = {n : n mod M = m}."""
    return [np.arange(m, n_angles, n_subsets, dtype=np.int32) for m in range(n_subsets)]


def poisson_gradient(geom: Geometry, f, g, mu=None, s=None, idx=None):
    """Table 1, PoissonLogLikelihood: H^T (g / (H f + s)) - H^T 1 on the rows idx.

    The ratio is taken as 0 where the expected projection H f + s is not
    positive.  Returns (gradient, H^T 1)."""
    ix = _idx(geom, idx)
    sens = back(geom, np.ones(geom.proj_shape), mu, ix)
    return _gradient_with_sens(geom, f, g, mu, s, ix, sens)


def osem(geom: Geometry, g, mu=None, n_iters: int = 1, n_subsets: int = 1, s=None, f0=None,
         callback=None) -> np.ndarray:
    """OSEM as Eq. 5 with the Table 1 preconditioner C = f / (H^(n)T 1), V = 0.

    f^(n+1) = f^(n) + f^(n) / sens_m * (H_m^T (g_m / (H_m f^(n) + s_m)) - sens_m)
    over subiterations n, with subset m = n mod M and sens_m = H_m^T 1.  Where
    sens_m = 0 the voxel keeps its value.
    """
    f = np.ones(geom.object_shape) if f0 is None else np.array(f0, dtype=np.float64)
    subs = subsets(geom.n_angles, n_subsets)
    sens = [back(geom, np.ones(geom.proj_shape), mu, ix) for ix in subs]
    for it in range(n_iters):
        for m, ix in enumerate(subs):
            grad, _ = _gradient_with_sens(geom, f, g, mu, s, ix, sens[m])
            pos = sens[m] > 0
            step = np.zeros_like(f)
            step[pos] = f[pos] / sens[m][pos] * grad[pos]
            f = f + step
            if callback is not None:
                callback(it, m, f)
    return f


def _gradient_with_sens(geom, f, g, mu, s, ix, sens):
    gbar = forward(geom, f, mu, ix)
    if s is not None:
        gbar[ix] += np.asarray(s, np.float64)[ix]
    q = np.zeros(geom.proj_shape)
    gi = np.asarray(g, np.float64)[ix]
    ei = gbar[ix]
    q[ix] = np.where(ei > 0, gi / np.where(ei > 0, ei, 1.0), 0.0)
    return back(geom, q, mu, ix) - sens, sens


def dense_matrix(geom: Geometry, mu=None, idx=None) -> np.ndarray:
    """H as a (A*N*Nz) x (N*N*Nz) matrix, by projecting every unit vector."""
    nobj = int(np.prod(geom.object_shape))
    cols = []
    for q in range(nobj):
        e = np.zeros(nobj)
        e[q] = 1.0
        cols.append(forward(geom, e.reshape(geom.object_shape), mu, idx).ravel())
    return np.stack(cols, axis=1)


def log_likelihood(geom: Geometry, f, g, mu=None, s=None, idx=None) -> float:
    """Poisson log-likelihood sum(g log(Hf+s) - (Hf+s)) over rows idx."""
    ix = _idx(geom, idx)
    gbar = forward(geom, f, mu, ix)[ix]
    if s is not None:
        gbar = gbar + np.asarray(s, np.float64)[ix]
    gi = np.asarray(g, np.float64)[ix]
    return float(np.sum(np.where(gi > 0, gi * np.log(np.maximum(gbar, 1e-300)), 0.0) - gbar))


def unrolled_osem_grad(geom: Geometry, g, f0, target, n_steps: int, n_subsets: int, mu=None,
                       s=None):
    """Loss L = sum((f_K - target)^2) / n_voxels after K = n_steps OSEM
    subiterations from f0 (subiteration k uses subset k mod M, the update of
    ``osem`` in its multiplicative form f * H_m^T q / sens_m), and dL/df0.

    Reverse mode, written out: with q_k = g / ghat_k (0 where ghat_k <= 0),
    ghat_k = H_m f_k + s, b_k = H_m^T q_k and f_(k+1) = f_k b_k / sens_m where
    sens_m > 0 (else f_k), an adjoint gbar = dL/df_(k+1) gives
        u = gbar f_k / sens_m           (dL/db_k, 0 where sens_m = 0)
        v = H_m u                       (dL/dq_k)
        w = -v g / ghat_k^2             (dL/dghat_k, 0 where ghat_k <= 0)
        dL/df_k = gbar b_k / sens_m + H_m^T w   (gbar where sens_m = 0).
    Returns (L, dL/df0)."""
    subs = subsets(geom.n_angles, n_subsets)
    sens = [back(geom, np.ones(geom.proj_shape), mu, ix) for ix in subs]
    g = np.asarray(g, np.float64)
    f = np.array(f0, dtype=np.float64)
    tape = []
    for k in range(n_steps):
        m = k % n_subsets
        ix = subs[m]
        ghat = forward(geom, f, mu, ix)
        if s is not None:
            ghat[ix] += np.asarray(s, np.float64)[ix]
        pos_g = np.zeros(geom.proj_shape, dtype=bool)
        pos_g[ix] = ghat[ix] > 0
        q = np.zeros(geom.proj_shape)
        q[pos_g] = g[pos_g] / ghat[pos_g]
        b = back(geom, q, mu, ix)
        pos = sens[m] > 0
        f1 = f.copy()
        f1[pos] = f[pos] * b[pos] / sens[m][pos]
        tape.append((m, f, ghat, pos_g, b))
        f = f1
    n_vox = f.size
    diff = f - np.asarray(target, np.float64)
    loss = float(np.sum(diff * diff) / n_vox)
    gbar = 2.0 * diff / n_vox
    for m, fk, ghat, pos_g, b in reversed(tape):
        ix = subs[m]
        pos = sens[m] > 0
        u = np.zeros(geom.object_shape)
        u[pos] = gbar[pos] * fk[pos] / sens[m][pos]
        v = forward(geom, u, mu, ix)
        w = np.zeros(geom.proj_shape)
        w[pos_g] = -v[pos_g] * g[pos_g] / (ghat[pos_g] * ghat[pos_g])
        prev = gbar.copy()
        prev[pos] = gbar[pos] * b[pos] / sens[m][pos]
        gbar = prev + back(geom, w, mu, ix)
    return loss, gbar


# ------------------------------------------------ BSREM with the RDP prior --
#
# Section 2.1.3: Eq. 4 with the Table 1 BSREM preconditioner
#     C = f alpha^(n) / (c^(n) H^T 1),   beta^(n) = c^(n) beta,
# and the relative difference prior of Table 1,
#     V(f) = sum_r sum_{s in N(r)} w_rs phi(f_r, f_s),
#     phi(a, b) = (a - b)^2 / (a + b + gamma |a - b|).
# Readings where the paper is silent: N(r) = the 26 neighbours of voxel r
# inside the grid, w_rs = 1 / (Euclidean distance in voxels); c^(n) = the
# subset's share of the angles; H^T 1 in C is the all-angle sensitivity;
# alpha^(n) = 1 / (1 + k) in iteration k = floor(n / M); phi and its
# derivative are 0 where a + b + gamma |a - b| = 0; after each update the
# image is clipped at 0 (the non-negativity BSREM maintains); voxels with
# zero sensitivity keep their value.

def _neighbour_offsets():
    offs = []
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                if dx or dy or dz:
                    offs.append((dx, dy, dz, 1.0 / np.sqrt(dx * dx + dy * dy + dz * dz)))
    return offs


def _pairs(f, dx, dy, dz):
    """Views (f_r, f_s) over all voxels r whose neighbour s = r + (dx,dy,dz) is inside."""
    def sl(d, n):
        return (slice(0, n - d), slice(d, n)) if d >= 0 else (slice(-d, n), slice(0, n + d))
    (ax, bx), (ay, by), (az, bz) = sl(dx, f.shape[0]), sl(dy, f.shape[1]), sl(dz, f.shape[2])
    return (ax, ay, az), (bx, by, bz)


def rdp_value(f, gamma: float) -> float:
    """V(f) of the relative difference prior, summed over ordered neighbour pairs."""
    f = np.asarray(f, np.float64)
    total = 0.0
    for dx, dy, dz, w in _neighbour_offsets():
        r, s = _pairs(f, dx, dy, dz)
        a, b = f[r], f[s]
        d = a - b
        den = a + b + gamma * np.abs(d)
        total += w * float(np.sum(np.where(den > 0, d * d / np.where(den > 0, den, 1.0), 0.0)))
    return total


def rdp_gradient(f, gamma: float) -> np.ndarray:
    """dV/df_r = 2 sum_s w_rs dphi/da(f_r, f_s) (phi is symmetric, so each
    ordered pair contributes the same derivative to both of its voxels), with
    dphi/da(a, b) = (a - b)(a + 3b + gamma |a - b|) / (a + b + gamma |a - b|)^2."""
    f = np.asarray(f, np.float64)
    grad = np.zeros_like(f)
    for dx, dy, dz, w in _neighbour_offsets():
        r, s = _pairs(f, dx, dy, dz)
        a, b = f[r], f[s]
        d = a - b
        den = a + b + gamma * np.abs(d)
        grad[r] += 2.0 * w * np.where(den > 0, d * (a + 3 * b + gamma * np.abs(d)) /
                                      np.where(den > 0, den * den, 1.0), 0.0)
    return grad


def bsrem(geom: Geometry, g, mu=None, n_iters: int = 1, n_subsets: int = 1, beta: float = 0.3,
          gamma: float = 2.0, s=None, f0=None, relaxation=None, callback=None) -> np.ndarray:
    """BSREM with the RDP prior, Eq. 4 with the Table 1 preconditioner:
    f <- max(0, f + f alpha / (c S) (H_m^T(g_m / (H_m f + s_m)) - H_m^T 1 - c beta grad V(f)))
    with S = H^T 1 over all angles and c = |S_m| / A; voxels with S = 0 keep
    their value.  relaxation(k) gives alpha for iteration k (default 1/(1+k))."""
    relaxation = relaxation or (lambda k: 1.0 / (1.0 + k))
    f = np.ones(geom.object_shape) if f0 is None else np.array(f0, dtype=np.float64)
    subs = subsets(geom.n_angles, n_subsets)
    sens = [back(geom, np.ones(geom.proj_shape), mu, ix) for ix in subs]
    s_all = np.sum(sens, axis=0)
    pos = s_all > 0
    for it in range(n_iters):
        alpha = relaxation(it)
        for m, ix in enumerate(subs):
            c = len(ix) / geom.n_angles
            grad, _ = _gradient_with_sens(geom, f, g, mu, s, ix, sens[m])
            step = grad - c * beta * rdp_gradient(f, gamma)
            f1 = f.copy()
            f1[pos] = np.maximum(0.0, f[pos] + f[pos] * alpha / (c * s_all[pos]) * step[pos])
            f = f1
            if callback is not None:
                callback(it, m, f)
    return f
