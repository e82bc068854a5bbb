"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: a special
case that reduces to a textbook or library routine, a closed form, an
invariant, or brute force on a tiny grid.  The readings of the paper that the
oracle follows (bilinear rotation about the grid centre, detector beyond the
+x end of the rotated depth axis, midpoint attenuation path, sampled
unit-sum Gaussian collimator response, interleaved subsets) are what is being
pinned where the paper itself does not fix the discretisation.
"""
import numpy as np
import pytest
import scipy.ndimage
import torch

from oracle import oracle as O
from paper_2309_01977_amd import phantoms as P


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------- P1, P2 ----

def test_p1_zero_angle_is_plain_sum_along_x():
    """Eq. 1 at angle 0 without attenuation or blur: P_x sums along x."""
    g = O.Geometry(9, 5, 1, 0.5)
    f = rng(1).random((9, 9, 5))
    p = O.forward(g, f)
    np.testing.assert_allclose(p[0], f.sum(axis=0), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n", [8, 9])
def test_p2_right_angles_are_permutations(n):
    """At 90, 180, 270 degrees the bilinear rotation is a pure permutation:
    the detector at 90 degrees faces +y, so the projection sums along y
    with the bin axis reversed in x, and so on (counter-clockwise gantry)."""
    g = O.Geometry(n, 4, 4, 0.4)
    f = rng(2).random((n, n, 4))
    p = O.forward(g, f)
    np.testing.assert_allclose(p[0], f.sum(axis=0), rtol=1e-14)
    np.testing.assert_allclose(p[1], f.sum(axis=1)[::-1, :], rtol=1e-14)
    np.testing.assert_allclose(p[2], f.sum(axis=0)[::-1, :], rtol=1e-14)
    np.testing.assert_allclose(p[3], f.sum(axis=1), rtol=1e-14)
    # the rotated volume at 90 degrees is np.rot90 of each axial slice
    rot = O.rotate(f, 90.0)
    for ip in range(n):
        for jp in range(n):
            np.testing.assert_array_equal(rot[ip, jp], f[n - 1 - jp, ip])


# ------------------------------------------------------------------- P3 ----

@pytest.mark.parametrize("deg", [17.0, 33.3, 123.0, 251.5])
def test_p3_rotation_matches_grid_sample_and_its_autograd_transpose(deg):
    """T_rot against torch grid_sample (bilinear, zero padding,
    align_corners=True) in float64, and T_rot^T against autograd of the same
    call, which is its exact transpose."""
    n, nz = 11, 3
    f = rng(3).random((n, n, nz))
    ours = O.rotate(f, deg)
    c = 0.5 * (n - 1)
    cs, sn = np.cos(np.deg2rad(deg)), np.sin(np.deg2rad(deg))
    ip, jp = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    X = c + cs * (ip - c) - sn * (jp - c)
    Y = c + sn * (ip - c) + cs * (jp - c)
    # image rows = y (height), columns = x (width); grid[..., 0] = x
    img = torch.tensor(f.transpose(2, 1, 0)[None], dtype=torch.float64, requires_grad=True)
    grid = torch.tensor(np.stack([2 * X / (n - 1) - 1, 2 * Y / (n - 1) - 1], -1)[None],
                        dtype=torch.float64)
    out = torch.nn.functional.grid_sample(img, grid, mode="bilinear", padding_mode="zeros",
                                          align_corners=True)
    ref = out[0].permute(1, 2, 0).detach().numpy()  # [i'][j'][k]
    np.testing.assert_allclose(ours, ref, rtol=1e-13, atol=1e-13)
    w = rng(4).standard_normal((n, n, nz))
    out.backward(torch.tensor(w.transpose(2, 0, 1)[None], dtype=torch.float64))
    adj_ref = img.grad[0].numpy().transpose(2, 1, 0)
    np.testing.assert_allclose(O.rotate_adjoint(w, deg), adj_ref, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------- P4 ----

@pytest.mark.parametrize("n,nz,A,with_mu,psf", [(5, 3, 4, True, True), (6, 4, 5, True, True),
                                                (4, 2, 6, False, True), (7, 2, 3, True, False)])
def test_p4_dense_transpose_nonnegative_linear(n, nz, A, with_mu, psf):
    """Brute force: build H column by column; the oracle's back projection
    equals H^T, H >= 0, and the forward projection is linear."""
    r = rng(5)
    g = O.Geometry(n, nz, A, 0.7, *(0.05, 0.4) if psf else (0.0, 0.0),
                   angles_deg=list(r.uniform(0, 360, A)))
    mu = r.random((n, n, nz)) * 0.3 if with_mu else None
    H = O.dense_matrix(g, mu)
    assert H.min() >= 0
    y = r.standard_normal(g.proj_shape)
    np.testing.assert_allclose(O.back(g, y, mu).ravel(), H.T @ y.ravel(), rtol=1e-12, atol=1e-12)
    x1, x2 = r.standard_normal((2,) + g.object_shape)
    np.testing.assert_allclose(O.forward(g, 2 * x1 - 3 * x2, mu),
                               2 * O.forward(g, x1, mu) - 3 * O.forward(g, x2, mu), atol=1e-11)
    idx = [1, 2]
    Hs = O.dense_matrix(g, mu, idx)
    rows = np.zeros(g.proj_shape, bool)
    rows[idx] = True
    np.testing.assert_allclose(Hs[rows.ravel()], H[rows.ravel()], rtol=1e-14)
    assert not Hs[~rows.ravel()].any()


# ------------------------------------------------------------------- P5 ----

@pytest.mark.parametrize("deg,axis,near_end", [(0.0, 0, True), (90.0, 1, True), (180.0, 0, False)])
def test_p5_attenuation_closed_form(deg, axis, near_end):
    """Uniform mu everywhere, activity a in a run of voxels along the ray,
    no blur: each voxel is attenuated by exp(-mu dx (t + 1/2)) where t counts
    the voxels between it and the detector, a geometric series."""
    n, nz, dx, mu0, a = 12, 2, 0.48, 0.15, 3.0
    g = O.Geometry(n, nz, 1, dx, angles_deg=[deg])
    f = np.zeros((n, n, nz))
    i0, i1, lane = 2, 6, 5
    sl = [lane, lane, slice(None)]
    sl[axis] = slice(i0, i1 + 1)
    f[tuple(sl)] = a
    mu = np.full((n, n, nz), mu0)
    p = O.forward(g, f, mu)[0]
    q = np.exp(-mu0 * dx)
    cnt = i1 - i0 + 1
    t0 = (n - 1 - i1) if near_end else i0          # voxels between the run and the detector
    expect = a * np.exp(-mu0 * dx / 2) * q ** t0 * (1 - q ** cnt) / (1 - q)
    bin_ = {0.0: lane, 90.0: n - 1 - lane, 180.0: n - 1 - lane}[deg]
    np.testing.assert_allclose(p[bin_], expect, rtol=1e-13)
    assert np.abs(np.delete(p, bin_, axis=0)).max() == 0


# ------------------------------------------------------------------- P6 ----

def _gauss_taps(sigma_px, K):
    m = np.arange(-K, K + 1)
    w = np.exp(-m ** 2 / (2 * sigma_px ** 2))
    return w / w.sum()


@pytest.mark.parametrize("depth", [2, 10, 20])
def test_p6_point_source_blur_width_and_position(depth):
    """A point source at rotated depth i' projects to the outer product of the
    sampled Gaussian g_i' centred on its (bin, slice); the width follows
    sigma = a d + b with d measured from the detector face at the +x end."""
    n, nz, dx = 24, 21, 0.48
    a, b = 0.03, 0.1
    g = O.Geometry(n, nz, 1, dx, a, b)
    f = np.zeros((n, n, nz))
    j0, k0 = 11, 10
    f[depth, j0, k0] = 1.0
    p = O.forward(g, f)[0]
    c = 0.5 * (n - 1)
    d = n * dx / 2 - (depth - c) * dx
    s = (a * d + b) / dx
    K = int(np.ceil(4 * s - 1e-9))
    k1 = _gauss_taps(s, K)
    expect = np.zeros((n, nz))
    expect[j0 - K:j0 + K + 1, k0 - K:k0 + K + 1] = np.outer(k1, k1)
    np.testing.assert_allclose(p, expect, rtol=1e-12, atol=1e-15)
    assert abs(p.sum() - 1) < 1e-12


def test_p6_each_angle_blurs_with_its_own_detector_distance():
    """A point source seen at 0, 90, 180 and 270 degrees (exact permutations,
    R3) with a different detector radius per angle: projection n is the
    sampled Gaussian of sigma = a d_n + b, d_n = max(0, R_n - (i'_n - c) dx),
    centred on the point's rotated (bin, slice), cut at the detector edge
    (zero padding, R7).  The 2 cm radius puts the point beyond the detector
    face at 0 degrees (d clamped to 0, R6); at 270 degrees the kernel runs
    past the last bin."""
    n, nz, dx, a, b = 24, 21, 0.48, 0.03, 0.1
    radii = [2.0, 15.0, 22.0, 30.0]
    g = O.Geometry(n, nz, 4, dx, a, b, 4.0, [0.0, 90.0, 180.0, 270.0], radii)
    x0, y0, k0 = 16, 12, 10
    f = np.zeros((n, n, nz))
    f[x0, y0, k0] = 1.0
    p = O.forward(g, f)
    c = 0.5 * (n - 1)
    # rotated (depth, bin) of object voxel (x0, y0): inverse of the R3 map
    hits = [(x0, y0), (y0, n - 1 - x0), (n - 1 - x0, n - 1 - y0), (n - 1 - y0, x0)]
    widths = []
    for m, ((ip, jp), R) in enumerate(zip(hits, radii)):
        d = max(0.0, R - (ip - c) * dx)
        s = (a * d + b) / dx
        K = int(np.ceil(4 * s - 1e-9))
        k1 = _gauss_taps(s, K)
        big = np.zeros((n + 2 * K, nz + 2 * K))
        big[jp:jp + 2 * K + 1, k0:k0 + 2 * K + 1] = np.outer(k1, k1)
        expect = big[K:K + n, K:K + nz]
        np.testing.assert_allclose(p[m], expect, rtol=1e-12, atol=1e-15, err_msg=f"angle {m}")
        widths.append(K)
    assert widths[0] == 1 and jp + widths[3] > n - 1  # the clamp and the edge are exercised
    assert p[3].sum() < 1 - 1e-5  # the tail past the last bin is lost


def test_repeated_angles_project_once_and_back_project_per_occurrence():
    """An angle listed twice: the forward's rows are a set (the row equals the
    one projected alone, whatever the thread schedule), the back projection
    is a sum over list entries (linearity: twice that angle's term)."""
    g = O.Geometry(12, 5, 6, 0.5, 0.03, 0.1)
    r = rng(41)
    f, y, mu = r.random(g.object_shape), r.random(g.proj_shape), 0.1 * r.random(g.object_shape)
    np.testing.assert_array_equal(O.forward(g, f, mu, [3, 3, 5]), O.forward(g, f, mu, [3, 5]))
    np.testing.assert_array_equal(O.forward(g, f, mu, [5, 3, 3, 3]), O.forward(g, f, mu, [3, 5]))
    b = O.back(g, y, mu, [3, 3, 5])
    np.testing.assert_allclose(b, 2 * O.back(g, y, mu, [3]) + O.back(g, y, mu, [5]), rtol=1e-13, atol=1e-15)


def test_p6_second_moment_matches_sigma_squared():
    """Second moment of the discrete kernel equals sigma(d)^2 within 0.2 %
    where sigma is at least one pixel (closed form of the continuous
    Gaussian; the truncation at 4 sigma and the sampling cost < 0.2 %)."""
    n, dx, a, b = 128, 0.48, 0.03, 0.1
    g = O.Geometry(n, 4, 1, dx, a, b)
    c = 0.5 * (n - 1)
    checked = 0
    for ip in range(n):
        d = n * dx / 2 - (ip - c) * dx
        s = (a * d + b) / dx
        if s < 1.0:
            continue
        t = O.psf_taps(g, ip)
        K = len(t) - 1
        full = np.concatenate([t[:0:-1], t])
        m = np.arange(-K, K + 1)
        assert abs(full.sum() - 1) < 1e-14
        assert abs((full * m ** 2).sum() / s ** 2 - 1) < 2e-3
        checked += 1
    assert checked > 20


def test_p6_blur_equals_library_2d_convolution():
    """A single depth plane of random activity: the oracle's blur equals
    scipy.ndimage.convolve with the 2D outer-product kernel and zero
    padding (cval 0), summed over the one occupied depth."""
    n, nz, dx = 20, 17, 0.48
    g = O.Geometry(n, nz, 1, dx, 0.03, 0.1)
    f = np.zeros((n, n, nz))
    depth = 4
    plane = rng(6).random((n, nz))
    f[depth] = plane
    p = O.forward(g, f)[0]
    t = O.psf_taps(g, depth)
    k1 = np.concatenate([t[:0:-1], t])
    ref = scipy.ndimage.convolve(plane, np.outer(k1, k1), mode="constant", cval=0.0)
    np.testing.assert_allclose(p, ref, rtol=1e-12, atol=1e-14)


# ------------------------------------------------- Eq. 1 operator order ----
#
# Eq. 1 applies T_att before T_cdr.  At 0 and 90 degrees the rotation is an
# exact permutation (R3), so with an absorber that covers only part of the
# detector bins every value below is a closed form: the sampled Gaussian of
# the source depth (R6, R7) times exp(-mu dx (t + 1/2)), t being the voxels
# between the emitting voxel and the detector (R5).  Blurring first and
# attenuating afterwards would attenuate each blurred bin by its own ray, so
# the bins beyond the absorber edge would come out unattenuated.

def _rot_to_obj(deg, n):
    """Object (x, y) of rotated-frame (depth i', bin j') at 0 or 90 degrees."""
    return (lambda i, j: (i, j)) if deg == 0.0 else (lambda i, j: (n - 1 - j, i))


def _half_absorber(deg, n, nz, mu0, j_edge):
    """mu0 on every rotated ray with bin j' <= j_edge (all depths, all
    slices), 0 on the others."""
    to_obj = _rot_to_obj(deg, n)
    mu = np.zeros((n, n, nz))
    for i in range(n):
        for j in range(j_edge + 1):
            mu[to_obj(i, j)] = mu0
    return mu


def _depth_taps(n, dx, a, b, depth):
    c = 0.5 * (n - 1)
    s = (a * (n * dx / 2 - (depth - c) * dx) + b) / dx
    K = int(np.ceil(4 * s - 1e-9))
    return _gauss_taps(s, K), K


@pytest.mark.parametrize("deg", [0.0, 90.0])
def test_eq1_point_source_is_attenuated_once_then_blurred(deg):
    """Forward: a point source at rotated (depth 4, bin 11, slice 7), with
    the absorber covering bins 0..11, projects to exp(-tau of the source)
    times g_4 (x) g_4 centred on (bin 11, slice 7); half of the kernel lies
    on bins outside the absorber and still carries the source's factor."""
    n, nz, dx, mu0, a, b = 24, 15, 0.48, 0.15, 0.03, 0.1
    ip, jp, k0 = 4, 11, 7
    g = O.Geometry(n, nz, 1, dx, a, b, angles_deg=[deg])
    to_obj = _rot_to_obj(deg, n)
    f = np.zeros((n, n, nz))
    f[to_obj(ip, jp) + (k0,)] = 1.0
    mu = _half_absorber(deg, n, nz, mu0, jp)
    p = O.forward(g, f, mu)[0]
    k1, K = _depth_taps(n, dx, a, b, ip)
    assert K == 4
    att = np.exp(-mu0 * dx * ((n - 1 - ip) + 0.5))
    expect = np.zeros((n, nz))
    expect[jp - K:jp + K + 1, k0 - K:k0 + K + 1] = att * np.outer(k1, k1)
    np.testing.assert_allclose(p, expect, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("deg", [0.0, 90.0])
def test_eq1_back_projection_blurs_then_attenuates_by_the_voxel_ray(deg):
    """Back projection (the transpose, applied in reverse order): a unit
    count in (bin 11, slice 7) reaches the voxel at rotated (i', j', k) as
    g_i'(j' - 11) g_i'(k - 7) times the attenuation factor of that voxel's
    own ray: exp(-mu dx (N - 1 - i' + 1/2)) for j' <= 11 inside the
    absorber, 1 beyond its edge."""
    n, nz, dx, mu0, a, b = 24, 15, 0.48, 0.15, 0.03, 0.1
    jp, k0 = 11, 7
    g = O.Geometry(n, nz, 1, dx, a, b, angles_deg=[deg])
    to_obj = _rot_to_obj(deg, n)
    mu = _half_absorber(deg, n, nz, mu0, jp)
    y = np.zeros(g.proj_shape)
    y[0, jp, k0] = 1.0
    out = O.back(g, y, mu)
    expect = np.zeros((n, n, nz))
    for i in range(n):
        k1, K = _depth_taps(n, dx, a, b, i)
        for m in range(-K, K + 1):
            j = jp + m
            if not 0 <= j < n:
                continue
            att = np.exp(-mu0 * dx * ((n - 1 - i) + 0.5)) if j <= jp else 1.0
            lo, hi = max(0, k0 - K), min(nz, k0 + K + 1)
            expect[to_obj(i, j) + (slice(lo, hi),)] = att * k1[K + m] * k1[K + lo - k0:K + hi - k0]
    assert (expect > 0).sum() > 300
    np.testing.assert_allclose(out, expect, rtol=1e-12, atol=1e-15)


# ------------------------------------------------------------------- P7 ----

def _bin_chord(v_lo, v_hi, rho):
    """Integral of the chord 2 sqrt(rho^2 - v^2) over [v_lo, v_hi]."""
    def F(y):
        y = np.clip(y, -rho, rho)
        return y * np.sqrt(rho * rho - y * y) + rho * rho * np.arcsin(y / rho)
    return F(v_hi) - F(v_lo)


@pytest.mark.parametrize("deg", [0.0, 30.0, 90.0, 200.0])
def test_p7_off_centre_disc_projects_to_its_chord_profile(deg):
    """An off-centre uniform cylinder (axis along z) projects, at every angle,
    to the chord profile of a disc centred at detector coordinate
    v0 = -sin(t) x0 + cos(t) y0.  At 0 and 90 degrees only the voxelisation
    differs from the bin-averaged chord; at oblique angles the bilinear
    resampling smooths the edges, so interior bins are compared."""
    n, nz, dx, rho = 64, 2, 0.48, 5.0
    x0, y0 = 7.0, 3.0
    f = P.voxelise([P.Shape("cylinder", (x0, y0, 0.0), (rho, 100.0), 1.0)], n, nz, dx, ss=8)
    g = O.Geometry(n, nz, 1, dx, angles_deg=[deg])
    p = O.forward(g, f)[0][:, 0]
    t = np.deg2rad(deg)
    v0 = -np.sin(t) * x0 + np.cos(t) * y0
    c = 0.5 * (n - 1)
    v = (np.arange(n) - c) * dx
    expect = _bin_chord(v - dx / 2 - v0, v + dx / 2 - v0, rho) / dx ** 2
    interior = np.abs(v - v0) < rho - 3 * dx
    rel = np.abs(p[interior] - expect[interior]) / expect[interior]
    tol = 5e-3 if deg in (0.0, 90.0) else 2e-2
    assert rel.max() < tol, rel.max()
    assert abs(p.sum() - expect.sum()) / expect.sum() < 1e-3
    outside = np.abs(v - v0) > rho + 2 * dx
    assert np.abs(p[outside]).max() < 1e-12


# ------------------------------------------------------------------- P8 ----

@pytest.mark.parametrize("which", ["C1", "C2_eight_angles"])
def test_p8_adjoint_identity_full_size(which):
    """<H x, y> = <x, H^T y> at the full workload grids, signed and
    non-negative x, y."""
    r = rng(7)
    if which == "C1":
        w = P.C1
        g = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b)
        idx = None
        mu = None
    else:
        w = P.C2
        g = O.Geometry(w.n, w.nz, w.n_angles, w.voxel_cm, w.psf_a, w.psf_b)
        idx = np.arange(3, 120, 15)
        mu = P.random_mu(g.object_shape, r, 0.2).astype(np.float64)
    for signed in (True, False):
        x = P.random_object(g.object_shape, r, signed).astype(np.float64)
        y = P.random_object(g.proj_shape, r, signed).astype(np.float64)
        if idx is not None:
            mask = np.zeros(g.n_angles, bool)
            mask[idx] = True
            y[~mask] = 0
        hx = O.forward(g, x, mu, idx)
        hty = O.back(g, y, mu, idx)
        lhs, rhs = np.vdot(hx, y), np.vdot(x, hty)
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.abs(hx).ravel() @ np.abs(y).ravel())


# ------------------------------------------------------------------- P9 ----

def test_p9_half_turn_mirrors_the_projection():
    """Without attenuation or blur the samples at t + 180 degrees are those at
    t mirrored through the centre, so p_{t+180}[r] = p_t[N-1-r]."""
    n, nz = 15, 3
    ang = [23.0, 203.0, 71.5, 251.5]
    g = O.Geometry(n, nz, 4, 0.5, angles_deg=ang)
    f = rng(8).random((n, n, nz))
    p = O.forward(g, f)
    np.testing.assert_allclose(p[1], p[0][::-1], rtol=1e-13)
    np.testing.assert_allclose(p[3], p[2][::-1], rtol=1e-13)


# -------------------------------------------------------------- P10-P14 ----

def _small_problem(seed=9, n=16, nz=6, A=12, with_mu=True):
    r = rng(seed)
    g = O.Geometry(n, nz, A, 0.48, 0.03, 0.1)
    f_true = P.random_object(g.object_shape, r).astype(np.float64) + 0.5
    mu = P.random_mu(g.object_shape, r, 0.15).astype(np.float64) if with_mu else None
    gbar = O.forward(g, f_true, mu)
    data = P.poisson_counts(gbar, 2e5, r).astype(np.float64)
    return g, f_true, mu, data


def test_p10_osem_count_conservation():
    """After each subiteration sum_j sens_m,j f'_j = sum_{i in S_m, Hf>0} g_i:
    a property of the multiplicative update for any H and its transpose."""
    g, _, mu, data = _small_problem()
    subs = O.subsets(g.n_angles, 4)
    sens = [O.back(g, np.ones(g.proj_shape), mu, ix) for ix in subs]
    seen = []

    def cb(it, m, f):
        seen.append((m, f.copy()))

    O.osem(g, data, mu, n_iters=2, n_subsets=4, callback=cb)
    prev = np.ones(g.object_shape)
    for m, f in seen:
        gbar = O.forward(g, prev, mu, subs[m])[subs[m]]
        lhs = np.sum(sens[m] * f)
        rhs = np.sum(np.where(gbar > 0, data[subs[m]], 0))
        assert abs(lhs - rhs) <= 1e-12 * rhs
        prev = f


def test_p11_osem_fixed_point():
    """Noise-free data g = H f* and f0 = f* leave f unchanged."""
    g, f_true, mu, _ = _small_problem()
    data = O.forward(g, f_true, mu)
    f = O.osem(g, data, mu, n_iters=2, n_subsets=3, f0=f_true)
    np.testing.assert_allclose(f, f_true, rtol=1e-12)


def test_p12_mlem_likelihood_is_monotone():
    """With one subset (MLEM) the Poisson log-likelihood never decreases."""
    g, _, mu, data = _small_problem(n=12, nz=4, A=8)
    vals = []

    def cb(it, m, f):
        vals.append(O.log_likelihood(g, f, data, mu))

    O.osem(g, data, mu, n_iters=6, n_subsets=1, callback=cb)
    vals = [O.log_likelihood(g, np.ones(g.object_shape), data, mu)] + vals
    for a, b in zip(vals, vals[1:]):
        assert b >= a - 1e-12 * abs(a)
    assert vals[-1] > vals[0]


def test_p13_degenerate_identity_system():
    """N = 1, one angle, no attenuation or blur: H = I, and one OSEM step
    from f0 = 1 returns the data."""
    g = O.Geometry(1, 5, 1, 0.5)
    data = np.array([[[3.0, 0.0, 7.5, 1.0, 2.0]]])
    np.testing.assert_array_equal(O.forward(g, np.arange(5.0).reshape(1, 1, 5)),
                                  np.arange(5.0).reshape(1, 1, 5))
    f = O.osem(g, data, None, n_iters=1, n_subsets=1)
    np.testing.assert_allclose(f.ravel(), data.ravel(), rtol=1e-15)


def test_p14_gradient_form_equals_multiplicative_form():
    """Eq. 5 with the Table 1 preconditioner f / sens and the gradient
    H^T(g/Hf) - H^T 1 equals the multiplicative EM form f H^T(g/Hf) / sens."""
    g, _, mu, data = _small_problem()
    subs = O.subsets(g.n_angles, 3)
    f = O.osem(g, data, mu, n_iters=1, n_subsets=3)
    fm = np.ones(g.object_shape)
    for ix in subs:
        sens = O.back(g, np.ones(g.proj_shape), mu, ix)
        gbar = O.forward(g, fm, mu, ix)
        q = np.zeros(g.proj_shape)
        q[ix] = np.where(gbar[ix] > 0, data[ix] / np.where(gbar[ix] > 0, gbar[ix], 1), 0)
        b = O.back(g, q, mu, ix)
        fm = np.where(sens > 0, fm * b / np.where(sens > 0, sens, 1), fm)
    np.testing.assert_allclose(f, fm, rtol=1e-13)


def test_zero_sensitivity_voxels_keep_their_value():
    """A voxel that no ray of the subset reaches (a grid corner at 45 degrees)
    keeps its value (reading of the 0/0 case); every other voxel is updated."""
    g = O.Geometry(16, 2, 1, 0.5, angles_deg=[45.0])
    sens = O.back(g, np.ones(g.proj_shape), None)
    assert (sens == 0).any() and (sens > 0).any()
    data = rng(10).random(g.proj_shape) * 5 + 1
    f0 = np.full(g.object_shape, 2.0)
    f = O.osem(g, data, None, 1, 1, f0=f0)
    np.testing.assert_array_equal(f[sens == 0], 2.0)
    assert np.all(f[sens > 0] != 2.0)


# ---------------------------------------------- P15, P16: unrolled OSEM ----

def _unrolled_problem(seed=21):
    r = rng(seed)
    g = O.Geometry(5, 3, 6, 0.7, 0.05, 0.4, angles_deg=[0.0, 45.0, 100.0, 170.0, 225.0, 300.0])
    mu = r.random(g.object_shape) * 0.3
    f_true = r.random(g.object_shape) + 0.2
    data = O.forward(g, f_true, mu) * 3.0
    s = r.random(g.proj_shape) * 0.05
    f0 = r.random(g.object_shape) + 0.5
    target = r.random(g.object_shape)
    return g, mu, data, s, f0, target


@pytest.mark.parametrize("with_s", [False, True])
def test_p15_unrolled_osem_gradient_equals_autograd_of_dense_osem(with_s):
    """Brute force: OSEM written with the dense matrix H in float64 torch and
    differentiated by autograd gives the same loss and gradient as the
    oracle's hand-written reverse recursion (rays that miss the object give
    zero expected counts at 45 degrees, exercising the q = 0 branch)."""
    g, mu, data, s, f0, target = _unrolled_problem()
    s = s if with_s else None
    K, M = 5, 2
    loss, grad = O.unrolled_osem_grad(g, data, f0, target, K, M, mu, s)
    H = torch.from_numpy(O.dense_matrix(g, mu))
    A, n_bin = g.n_angles, g.proj_shape[1] * g.proj_shape[2]
    rows = [torch.from_numpy(np.repeat(np.isin(np.arange(A), ix), n_bin)) for ix in O.subsets(A, M)]
    gd = torch.from_numpy(data.ravel())
    sd = torch.zeros_like(gd) if s is None else torch.from_numpy(s.ravel())
    f = torch.from_numpy(f0.ravel()).clone().requires_grad_(True)
    x = f
    for k in range(K):
        Hm = H[rows[k % M]]
        sens = Hm.sum(0)
        ghat = Hm @ x + sd[rows[k % M]]
        q = torch.where(ghat > 0, gd[rows[k % M]] / torch.where(ghat > 0, ghat, torch.ones_like(ghat)),
                        torch.zeros_like(ghat))
        b = Hm.T @ q
        x = torch.where(sens > 0, x * b / torch.where(sens > 0, sens, torch.ones_like(sens)), x)
    L = ((x - torch.from_numpy(target.ravel())) ** 2).mean()
    L.backward()
    assert abs(L.item() - loss) <= 1e-12 * max(1.0, abs(loss))
    np.testing.assert_allclose(grad.ravel(), f.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_p16_unrolled_osem_gradient_matches_central_differences():
    """Directional derivatives of the unrolled loss by central differences in
    FP64 (eps 1e-5, error O(eps^2)) agree with the oracle gradient."""
    g, mu, data, s, f0, target = _unrolled_problem(22)
    K, M = 4, 3
    _, grad = O.unrolled_osem_grad(g, data, f0, target, K, M, mu, s)
    r = rng(23)
    for _ in range(3):
        v = r.standard_normal(g.object_shape)
        eps = 1e-5
        lp, _ = O.unrolled_osem_grad(g, data, f0 + eps * v, target, K, M, mu, s)
        lm, _ = O.unrolled_osem_grad(g, data, f0 - eps * v, target, K, M, mu, s)
        fd = (lp - lm) / (2 * eps)
        an = float(np.sum(grad * v))
        assert abs(fd - an) <= 1e-7 * abs(an) + 1e-12, (fd, an)


# ----------------------------------------- P17-P20: RDP prior and BSREM ----

def test_p17_rdp_gradient_matches_central_differences_of_the_prior():
    """The closed-form RDP gradient against central differences of V(f) as
    Table 1 defines it (FP64, eps 1e-6), at gamma 2 and 0."""
    r = rng(30)
    f = r.random((5, 4, 3)) + 0.1
    for gamma in (2.0, 0.0):
        grad = O.rdp_gradient(f, gamma)
        eps = 1e-6
        for q in r.choice(f.size, 12, replace=False):
            e = np.zeros(f.size)
            e[q] = eps
            e = e.reshape(f.shape)
            fd = (O.rdp_value(f + e, gamma) - O.rdp_value(f - e, gamma)) / (2 * eps)
            assert abs(fd - grad.ravel()[q]) <= 1e-7 * max(1.0, abs(fd)), (gamma, q)


def test_p18_rdp_hand_values_homogeneity_and_euler_identity():
    """Two voxels a = 1, b = 3, gamma = 2: V = 2 phi(1, 3) = 1 and dV/da =
    -0.875 (by hand).  phi is 1-homogeneous, so V(k f) = k V(f), the gradient
    is 0-homogeneous and <f, grad V(f)> = V(f) (Euler); a uniform image has
    zero gradient."""
    f2 = np.array([1.0, 3.0]).reshape(2, 1, 1)
    assert abs(O.rdp_value(f2, 2.0) - 1.0) < 1e-15
    assert abs(O.rdp_gradient(f2, 2.0)[0, 0, 0] + 0.875) < 1e-15
    r = rng(31)
    f = r.random((6, 5, 4)) + 0.05
    V, G = O.rdp_value(f, 2.0), O.rdp_gradient(f, 2.0)
    assert abs(np.sum(f * G) - V) <= 1e-12 * V
    assert abs(O.rdp_value(3.7 * f, 2.0) - 3.7 * V) <= 1e-12 * V
    np.testing.assert_allclose(O.rdp_gradient(3.7 * f, 2.0), G, rtol=1e-12, atol=1e-15)
    assert not O.rdp_gradient(np.full((4, 4, 4), 2.5), 2.0).any()


def test_p19_bsrem_without_prior_or_subsets_is_mlem():
    """One subset, beta = 0 and alpha = 1: the BSREM preconditioner f / H^T 1
    makes the update the MLEM (multiplicative EM) update of ``osem``."""
    g, _, mu, data = _small_problem()
    a = O.bsrem(g, data, mu, n_iters=3, n_subsets=1, beta=0.0, relaxation=lambda k: 1.0)
    b = O.osem(g, data, mu, n_iters=3, n_subsets=1)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_p20_bsrem_fixed_point_of_consistent_uniform_data():
    """Noise-free data of a uniform object: the object is a fixed point of
    BSREM-RDP with one subset (the likelihood gradient and the prior gradient
    both vanish there)."""
    g = O.Geometry(8, 4, 6, 0.6, 0.05, 0.3)
    fstar = np.full(g.object_shape, 2.0)
    data = O.forward(g, fstar)
    f = O.bsrem(g, data, None, n_iters=2, n_subsets=1, beta=0.3, gamma=2.0, f0=fstar)
    sens = O.back(g, np.ones(g.proj_shape), None)
    np.testing.assert_allclose(f[sens > 0], 2.0, rtol=1e-12)


def test_p18b_rdp_hot_voxel_closed_form():
    """One voxel of 1 in a zero 3x3x3 grid, gamma = 2: every pair with the
    centre has phi = 1/3 in both orders and all other pairs are 0, so
    V = 2 (6 + 12/sqrt 2 + 8/sqrt 3) / 3, and dV/df_centre = 2 sum w_s (1 * 3)/9."""
    f = np.zeros((3, 3, 3))
    f[1, 1, 1] = 1.0
    wsum = 6 + 12 / np.sqrt(2) + 8 / np.sqrt(3)
    assert abs(O.rdp_value(f, 2.0) - 2 * wsum / 3) < 1e-13
    assert abs(O.rdp_gradient(f, 2.0)[1, 1, 1] - 2 * wsum / 3) < 1e-13
    # a face neighbour b = 0 next to a = 1: dphi/db (b first) = (0 - 1)(0 + 3 + 2)/9, times 2 w = 2
    assert abs(O.rdp_gradient(f, 2.0)[0, 1, 1] - 2 * (-5 / 9)) < 1e-13


def test_p19b_bsrem_subset_scaling_on_a_symmetric_geometry():
    """Angles 0, 90, 180, 270 without attenuation or blur and two subsets
    {0, 180}, {90, 270}: every voxel's subset sensitivity is exactly half the
    total, so BSREM with beta = 0, alpha = 1 equals OSEM with two subsets, and
    one BSREM subiteration with the prior is that OSEM step minus
    f alpha beta grad V / H^T 1 (c cancels), clipped at 0."""
    g = O.Geometry(8, 3, 4, 0.6, angles_deg=[0.0, 90.0, 180.0, 270.0])
    r = rng(32)
    data = P.poisson_counts(O.forward(g, r.random(g.object_shape) + 0.5), 1e4, r).astype(np.float64)
    a = O.bsrem(g, data, None, n_iters=2, n_subsets=2, beta=0.0, relaxation=lambda k: 1.0)
    b = O.osem(g, data, None, n_iters=2, n_subsets=2)
    np.testing.assert_allclose(a, b, rtol=1e-12)
    f0 = r.random(g.object_shape) + 0.5
    beta, gamma, alpha = 0.3, 2.0, 0.7
    got = O.bsrem(g, data, None, n_iters=1, n_subsets=2, beta=beta, gamma=gamma, f0=f0,
                  relaxation=lambda k: alpha)
    S = O.back(g, np.ones(g.proj_shape), None)
    f = f0
    for ix in O.subsets(4, 2):
        Sm = O.back(g, np.ones(g.proj_shape), None, ix)
        gb = O.forward(g, f, None, ix)
        q = np.zeros(g.proj_shape)
        q[ix] = data[ix] / gb[ix]
        osem_step = f * O.back(g, q, None, ix) / Sm
        f = np.maximum(0.0, f + alpha * (osem_step - f) - f * alpha * beta * O.rdp_gradient(f, gamma) / S)
    np.testing.assert_allclose(got, f, rtol=1e-12)
