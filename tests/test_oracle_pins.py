"""Pins for the FP64 CPU oracle: closed forms, invariants, brute force, library
reductions and finite differences.  None of these re-types the oracle's own
formula; each would fail on a plausible mistake (a dropped term, a wrong sign
or index, a transposed operand).  CPU only."""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc
from synth.arch import ARCH_SMALL, Arch
from synth.params import init_params, mlp_layers
from synth.workloads import NEAR, FAR, nocs_affine, small_batch, uniform_xi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# helpers

def axis_rays(n, rng, lo=0.05, hi=0.95):
    """World rays along +x through the NOCS cube: o = (-1, y, z), d = (1, 0, 0).
    With x_nocs = x_world + 1/2 they enter at t = 1/2 and leave at t = 3/2."""
    yz = rng.uniform(lo, hi, (n, 2)) - 0.5
    o = np.concatenate([np.full((n, 1), -1.0), yz], 1).astype(np.float32)
    d = np.tile(np.array([1.0, 0.0, 0.0], np.float32), (n, 1))
    return o, d


def const_model(arch, sigma_log, table_value=1.0):
    """Parameters whose density is exp(sigma_log) and colour 0.5 everywhere:
    table entries all equal (every feature = table_value by partition of
    unity), W_1 = 1/in_dim so each hidden unit is table_value, deeper layers
    1/W, head row 0 = sigma_log / (W * table_value), colour rows 0."""
    p = np.zeros(arch.n_params, np.float32)
    p[:arch.n_table_params] = table_value
    off = arch.n_table_params
    for li, (o, i) in enumerate(arch.layer_shapes()):
        if li < arch.hidden:
            p[off:off + o * i] = 1.0 / i
        else:
            W = np.zeros((o, i), np.float32)
            W[0, :] = sigma_log / (i * table_value)
            p[off:off + o * i] = W.ravel()
        off += o * i
    return p


# --------------------------------------------------------------------------
# P1-P3: compositing

def test_p1_constant_density_transmittance_any_placement():
    """Constant density sigma0: T_final = exp(-sigma0 * sum(delta)) for any
    sample placement (the product of exp(-sigma0 delta_j) telescopes)."""
    arch = Arch(n_levels=4, log2_table=10, width=16, hidden=2)
    rng = np.random.default_rng(0)
    sigma_log = 2.0  # W_out row 0 = 2 / 16 = 1/8, exact
    p = const_model(arch, sigma_log)
    n, S = 64, 24
    o, d = axis_rays(n, rng)
    ray_obj = np.concatenate([o + 0.5, d], 1).astype(np.float32)
    t = np.sort(rng.uniform(0.5, 1.5, (n, S)), 1).astype(np.float32)
    dt = rng.uniform(0.0, 0.05, (n, S)).astype(np.float32)  # arbitrary placement
    flags = np.zeros(n, np.uint8)
    bg = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    out = orc.render_fwd(arch, p, ray_obj, t, dt, flags, bg=bg)
    sigma0 = math.exp(sigma_log)
    T_final = np.exp(-sigma0 * dt.astype(np.float64).sum(1))
    np.testing.assert_allclose(out["opacity"], 1.0 - T_final, rtol=0, atol=1e-13)
    # colour: 0.5 from the field plus the background through T_final
    expect = 0.5 * (1.0 - T_final)[:, None] + T_final[:, None] * bg
    np.testing.assert_allclose(out["rgb"], expect, rtol=0, atol=1e-13)


def test_p1_single_sample_depth():
    """One sample: D = (1 - exp(-sigma delta)) t."""
    rng = np.random.default_rng(1)
    n = 16
    sigma = rng.uniform(0.1, 30, (n, 1))
    dt = rng.uniform(0.001, 0.2, (n, 1))
    t = rng.uniform(0.5, 2.0, (n, 1))
    rgb = rng.uniform(0, 1, (n, 1, 3))
    out = orc.composite_fwd(sigma, rgb, t, dt, np.zeros((n, 3)))
    np.testing.assert_allclose(out["depth"], (1 - np.exp(-sigma * dt))[:, 0] * t[:, 0], rtol=1e-14)


def random_composite(rng, n=32, S=40):
    sigma = rng.exponential(5.0, (n, S))
    rgb = rng.uniform(0, 1, (n, S, 3))
    t = np.sort(rng.uniform(0.5, 2.5, (n, S)), 1)
    dt = np.diff(np.concatenate([t, np.full((n, 1), 2.5)], 1), axis=1)
    bg = rng.uniform(0, 1, (n, 3))
    return sigma, rgb, t, dt, bg


def test_p2_weights_sum_to_one_minus_final_transmittance():
    rng = np.random.default_rng(2)
    sigma, rgb, t, dt, bg = random_composite(rng)
    out = orc.composite_fwd(sigma, rgb, t, dt, bg)
    T_final = np.exp(-(sigma * dt).sum(1))
    np.testing.assert_allclose(out["w"].sum(1), 1.0 - T_final, atol=1e-14)
    np.testing.assert_allclose(out["opacity"], 1.0 - T_final, atol=1e-14)
    # each weight is the transmittance lost over its interval
    np.testing.assert_allclose(out["w"], out["T"][:, :-1] - out["T"][:, 1:], atol=1e-15)


def test_p3_composite_backward_closed_forms():
    rng = np.random.default_rng(3)
    sigma, rgb, t, dt, bg = random_composite(rng)
    n, S = sigma.shape
    out = orc.composite_fwd(sigma, rgb, t, dt, bg)
    T_final = out["T"][:, -1]
    z3, z1 = np.zeros((n, 3)), np.zeros(n)
    # d opacity / d sigma_j = delta_j T_final
    dsig, drgb = orc.composite_bwd(sigma, rgb, t, dt, bg, z3, z1, np.ones(n))
    np.testing.assert_allclose(dsig, dt * T_final[:, None], rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(drgb, 0.0)
    # d C_k / d c_jk = w_j
    for k in range(3):
        gC = np.zeros((n, 3))
        gC[:, k] = 1.0
        _, drgb = orc.composite_bwd(sigma, rgb, t, dt, bg, gC, z1)
        np.testing.assert_allclose(drgb[:, :, k], out["w"], rtol=1e-14)


def test_p3_composite_backward_finite_differences():
    rng = np.random.default_rng(4)
    sigma, rgb, t, dt, bg = random_composite(rng, n=8, S=12)
    n, S = sigma.shape
    gC = rng.normal(size=(n, 3))
    gD = rng.normal(size=n)
    gA = rng.normal(size=n)
    dsig, drgb = orc.composite_bwd(sigma, rgb, t, dt, bg, gC, gD, gA)

    def f(sig, col):
        o = orc.composite_fwd(sig, col, t, dt, bg)
        return (o["rgb"] * gC).sum(1) + o["depth"] * gD + o["opacity"] * gA

    h = 1e-6
    for j in range(S):
        e = np.zeros_like(sigma)
        e[:, j] = h
        fd = (f(sigma + e, rgb) - f(sigma - e, rgb)) / (2 * h)
        np.testing.assert_allclose(dsig[:, j], fd, rtol=1e-6, atol=1e-9)
        for k in range(3):
            e = np.zeros_like(rgb)
            e[:, j, k] = h
            fd = (f(sigma, rgb + e) - f(sigma, rgb - e)) / (2 * h)
            np.testing.assert_allclose(drgb[:, j, k], fd, rtol=1e-6, atol=1e-9)


# --------------------------------------------------------------------------
# P4-P7: sampler

def run_sampler(o, d, xi, prior, n_coarse=16, n_fine=48, include_coarse=False, eps=1e-4,
                near=0.0, far=10.0, uniform_only=False):
    return orc.sample(o, d, xi, n_coarse=n_coarse, n_fine=n_fine, include_coarse=include_coarse,
                      uniform_only=uniform_only, eps=eps, near=near, far=far,
                      world_to_obj=nocs_affine(), prior=prior)


@pytest.mark.parametrize("s", [1e-3, 0.37, 3.0, 41.0])
@pytest.mark.parametrize("dscale", [1.0, 4.0])
def test_p4_constant_prior_bins_closed_form(s, dscale):
    """Constant prior s: CDF_i = (1 - e^{-i tau}) / (1 - e^{-N_c tau}) with
    tau = s Delta |d|, so the first bin with CDF_{i+1} >= u is
    ceil(-ln(1 - u (1 - e^{-N_c tau})) / tau) - 1.  A world direction of
    length 4 (t in world units, NOCS length 4 per unit t) and the box given
    in the object frame by a 1/2 scale leave tau = s * 2 / N_c."""
    rng = np.random.default_rng(5)
    n, Nc, Nr = 256, 16, 48
    o, d = axis_rays(n, rng)
    d = d * np.float32(dscale)
    A = nocs_affine().reshape(3, 4).copy()
    if dscale != 1.0:
        A[:, :3] *= 0.5                       # x_nocs = x_world / 2 + 1/2
        o = o * np.float32(2.0)               # same NOCS entry point
    xi = uniform_xi(rng, n, Nr)
    prior = np.full((8, 8, 8), s, np.float32)
    out = orc.sample(o, d, xi, n_coarse=Nc, n_fine=Nr, include_coarse=False, uniform_only=False,
                     eps=1e-4, near=0.0, far=10.0, world_to_obj=A.ravel(), prior=prior)
    assert np.all(out["flags"] == 0)
    # |d_obj| = dscale * A-scale; t_f - t_n = 1 / |d_obj|; tau = s * (t_f - t_n)/N_c * |d_obj|
    tau = s * (1.0 / Nc)
    u = (np.arange(Nr)[None, :] + xi.astype(np.float64)) / Nr
    z = -np.log1p(-u * (-np.expm1(-Nc * tau))) / tau
    expect = np.ceil(z) - 1
    safe = np.abs(z - np.round(z)) > 1e-9
    assert safe.mean() > 0.99
    np.testing.assert_array_equal(out["bins"][safe], expect[safe].astype(np.int32))
    # each draw lies inside its bin, draws are sorted and inside [t_n, t_f]
    dl = dscale * (0.5 if dscale != 1.0 else 1.0)
    t = out["t"] * dl  # NOCS distance from the ray origin
    b = out["bins"]
    assert np.all(t >= 0.5 + b / Nc - 1e-14) and np.all(t <= 0.5 + (b + 1) / Nc + 1e-14)
    assert np.all(np.diff(t, axis=1) >= 0)
    np.testing.assert_allclose(out["dt"][:, -1], 1.5 - t[:, -1], atol=1e-14)


def test_p5_zero_prior_escapes_to_uniform():
    """All-zero prior: every ray escapes (sum rho_term = 0 < eps) and the
    draws are the stratified uniform ones, t_k = t_n + (k + xi_k)(t_f - t_n)/N_r."""
    rng = np.random.default_rng(6)
    n, Nc, Nr = 128, 16, 32
    o, d = axis_rays(n, rng)
    xi = uniform_xi(rng, n, Nr)
    out = run_sampler(o, d, xi, np.zeros((4, 4, 4), np.float32), Nc, Nr)
    assert np.all(out["flags"] == orc.FLAG_ESCAPED)
    assert np.all(out["bins"] == -1)
    expect = 0.5 + (np.arange(Nr)[None, :] + xi.astype(np.float64)) / Nr * 1.0
    np.testing.assert_allclose(out["t"], expect, rtol=0, atol=2e-16)


def test_p5_escape_threshold_is_strict():
    """Escape iff 1 - exp(-sum sigma delta) < eps: a constant prior s over a
    unit path has total 1 - e^{-s}; straddle eps."""
    rng = np.random.default_rng(7)
    n = 8
    o, d = axis_rays(n, rng)
    xi = uniform_xi(rng, n, 8)
    eps = 1e-3
    s_hit = -math.log1p(-eps) * 1.01
    s_esc = -math.log1p(-eps) * 0.99
    a = run_sampler(o, d, xi, np.full((4, 4, 4), s_hit, np.float32), 8, 8, eps=eps)
    b = run_sampler(o, d, xi, np.full((4, 4, 4), s_esc, np.float32), 8, 8, eps=eps)
    assert np.all(a["flags"] == 0) and np.all(b["flags"] == orc.FLAG_ESCAPED)


def test_p5_miss_rays():
    """Rays that do not meet the box: MISS, no samples."""
    o = np.array([[-1.0, 2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 5.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, 1.0]], np.float32)
    xi = np.full((3, 8), 0.5, np.float32)
    out = run_sampler(o, d, xi, np.ones((4, 4, 4), np.float32), 8, 8, near=0.1, far=3.0)
    # ray 0 passes beside the cube; ray 1 starts inside (hit); ray 2 points away
    assert out["flags"][0] == orc.FLAG_MISS and out["flags"][2] == orc.FLAG_MISS
    assert out["flags"][1] == 0
    assert np.all(out["t"][[0, 2]] == 0) and np.all(out["bins"][[0, 2]] == -1)


def test_p5_axis_parallel_rays_inside_and_outside_slab():
    """A direction component of exactly zero: the slab constrains nothing
    when the origin is inside it (including on its faces), rejects otherwise."""
    o = np.array([[-1.0, -0.5, 0.0], [-1.0, 0.5, 0.0], [-1.0, 0.50001, 0.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]] * 3, np.float32)
    out = run_sampler(o, d, np.full((3, 4), 0.5, np.float32), None, 4, 4, uniform_only=True)
    assert list(out["flags"]) == [orc.FLAG_UNIFORM, orc.FLAG_UNIFORM, orc.FLAG_MISS]


def test_p6_prior_trilinear_reproduces_affine_fields():
    """An affine field sampled on the vertices is reproduced exactly by
    trilinear interpolation; grid vertices return their stored values."""
    R = 5
    a = np.array([1.0, 2.0, 4.0])
    b = 0.5
    v = np.arange(R) / (R - 1)
    z, y, x = np.meshgrid(v, v, v, indexing="ij")
    grid = (a[0] * x + a[1] * y + a[2] * z + b).astype(np.float32)  # exact
    rng = np.random.default_rng(8)
    pts = rng.uniform(0, 1, (500, 3))
    np.testing.assert_allclose(orc.prior_lookup(grid, pts), pts @ a + b, rtol=0, atol=1e-14)
    vert = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    np.testing.assert_array_equal(orc.prior_lookup(grid, vert), grid.ravel().astype(np.float64))
    # outside [0,1] the lookup clamps to the boundary
    np.testing.assert_allclose(orc.prior_lookup(grid, np.array([[-1.0, 2.0, 0.5]])),
                               [a[1] + a[2] * 0.5 + b], atol=1e-14)


def test_p7_draws_follow_termination_pmf():
    """Chi-square test: the histogram of sampled bins follows
    rho_term,i / sum rho_term (Eq. (5), (6)) built here from the product form
    on the prior values at the coarse midpoints."""
    rng = np.random.default_rng(9)
    R, Nc, Nr = 16, 12, 32
    prior = rng.uniform(0.0, 20.0, (R, R, R)).astype(np.float32)
    n = 4000
    o = np.tile(np.array([[-1.0, 0.1, -0.2]], np.float32), (n, 1))
    d = np.tile(np.array([[1.0, 0.0, 0.0]], np.float32), (n, 1))
    xi = uniform_xi(rng, n, Nr)
    out = run_sampler(o, d, xi, prior, Nc, Nr)
    mids = 0.5 + (np.arange(Nc) + 0.5) / Nc
    pts = np.stack([mids - 0.5, np.full(Nc, 0.6), np.full(Nc, 0.3)], 1)
    sig = orc.prior_lookup(prior, pts)
    occ = 1.0 - np.exp(-sig / Nc)
    surv = np.concatenate([[1.0], np.cumprod(1.0 - occ)[:-1]])
    pmf = occ * surv
    pmf /= pmf.sum()
    counts = np.bincount(out["bins"].ravel(), minlength=Nc)
    exp_counts = pmf * counts.sum()
    keep = exp_counts > 5
    chi2 = (((counts - exp_counts) ** 2) / exp_counts)[keep].sum()
    dof = keep.sum() - 1
    # stratified draws have smaller variance than multinomial ones: 3 sigma bound
    assert chi2 < dof + 3 * math.sqrt(2 * dof), (chi2, dof)


def _edge_cdf(prior, pts, delta_nocs):
    """Eq. (6) CDF at the N_c + 1 bin edges, from the product form of Eq. (4)
    and (5) on the prior values at the bin midpoints (not the telescoped
    exponential form the oracle evaluates)."""
    sig = orc.prior_lookup(prior, pts)
    occ = 1.0 - np.exp(-sig * delta_nocs)
    surv = np.concatenate([[1.0], np.cumprod(1.0 - occ)[:-1]])
    term = occ * surv
    return np.concatenate([[0.0], np.cumsum(term) / term.sum()])


@pytest.mark.parametrize("dscale", [1.0, 3.0])
def test_p7_draw_position_inverts_piecewise_linear_cdf(dscale):
    """Inverse transform sampling on the discrete CDF (Sec. III-B), read as
    linear inside a bin: each draw t_k is the point where the piecewise-linear
    interpolation of the edge CDF reaches u_k = (k + xi_k)/N_r, so
    interp(t_k; edges, CDF) = u_k.  A bin midpoint, swapped bin endpoints or
    a shifted bin all fail this."""
    rng = np.random.default_rng(21)
    R, Nc, Nr, n = 16, 12, 40, 96
    prior = rng.uniform(0.0, 12.0, (R, R, R)).astype(np.float32)
    prior[:, :, : R // 3] = 0.0            # empty stretches: zero-mass bins
    o, d = axis_rays(n, rng)
    d = (d * np.float32(dscale)).astype(np.float32)
    xi = uniform_xi(rng, n, Nr)
    out = run_sampler(o, d, xi, prior, Nc, Nr)
    assert np.all(out["flags"] == 0)
    u = (np.arange(Nr)[None, :] + xi.astype(np.float64)) / Nr
    # world distance: the ray meets x_nocs = 0 at t = 1/(2|d|) and leaves at 3/(2|d|)
    tn, tf = 0.5 / dscale, 1.5 / dscale
    edges = tn + (tf - tn) * np.arange(Nc + 1) / Nc
    worst = 0.0
    for r in range(n):
        yz = o[r, 1:].astype(np.float64) + 0.5
        pts = np.stack([(np.arange(Nc) + 0.5) / Nc, np.full(Nc, yz[0]), np.full(Nc, yz[1])], 1)
        cdf = _edge_cdf(prior, pts, 1.0 / Nc)
        got = np.interp(out["t"][r], edges, cdf)
        worst = max(worst, float(np.abs(got - u[r]).max()))
    assert worst < 1e-12, worst


def test_p7_draw_position_small_prior_limit():
    """As a constant prior s -> 0 the CDF becomes i/N_c and the draws tend to
    the stratified uniform ones, t_k -> t_n + u_k (t_f - t_n), with an error
    of order s."""
    rng = np.random.default_rng(22)
    n, Nc, Nr = 64, 16, 48
    o, d = axis_rays(n, rng)
    xi = uniform_xi(rng, n, Nr)
    u = (np.arange(Nr)[None, :] + xi.astype(np.float64)) / Nr
    errs = []
    for s in (1e-2, 1e-3):
        out = run_sampler(o, d, xi, np.full((4, 4, 4), s, np.float32), Nc, Nr, eps=1e-6)
        assert np.all(out["flags"] == 0)
        e = np.abs(out["t"] - (0.5 + u)).max()
        assert e < s, (s, e)
        errs.append(e)
    assert errs[1] < errs[0] / 5  # the error shrinks with s


def test_sampler_merge_includes_coarse_midpoints():
    """With the coarse samples rendered, the sorted union of the N_c bin
    midpoints and the N_r draws is returned, with delta = next gap * |d|."""
    rng = np.random.default_rng(10)
    n, Nc, Nr = 64, 16, 48
    o, d = axis_rays(n, rng)
    d = d * 2.0  # |d| = 2 in world units -> NOCS length per unit t is 2
    prior = rng.uniform(0.01, 1.0, (16, 16, 16)).astype(np.float32)
    out = run_sampler(o, d, uniform_xi(rng, n, Nr), prior, Nc, Nr, include_coarse=True)
    t = out["t"]
    assert t.shape == (n, Nc + Nr)
    mids = 0.25 + (np.arange(Nc) + 0.5) * (0.5 / Nc)  # t_n = 1/4, t_f = 3/4
    for r in range(n):
        assert np.all(np.isin(mids, t[r]))
    assert np.all(np.diff(t, axis=1) >= 0)
    np.testing.assert_allclose(out["dt"][:, :-1], np.diff(t, axis=1) * 2.0, rtol=1e-15)
    np.testing.assert_allclose(out["dt"][:, -1], (0.75 - t[:, -1]) * 2.0, rtol=1e-14)


# --------------------------------------------------------------------------
# P8-P9: hash encoding

TINY = Arch(n_levels=3, log2_table=6, n_features=2, base_res=2, growth="2", width=16, hidden=1,
            resolutions=(2, 3, 5))


def exact_cell(x32, N):
    c = math.floor(Fraction(float(x32)) * N)
    return min(c, N - 1)


def hash_index(v, N, T):
    side = N + 1
    if side**3 <= T:
        return v[0] + side * (v[1] + side * v[2])
    return ((v[0] * 1) ^ (v[1] * 2654435761) ^ (v[2] * 805459861)) % 2**32 % T


def test_p8_hash_known_answer():
    """Corner (1, 1, 1) of a hashed level with T = 2^14:
    1 xor 2654435761 xor 805459861 = 3459891681 + ... ; mod 2^14 = 11813."""
    arch = Arch(n_levels=1, log2_table=14, width=16, hidden=1, resolutions=(40,))  # 41^3 > 2^14
    x = np.array([[1.5 / 40, 1.5 / 40, 1.5 / 40]], np.float32)  # cell (1,1,1)
    _, idx, _ = orc.encode(arch, np.zeros(arch.n_table_params, np.float32), x, with_corners=True)
    assert idx[0, 0, 0] == 11813


def test_p8_corner_indices_brute_force():
    rng = np.random.default_rng(11)
    T = TINY.table_size
    pts = rng.uniform(0, 1, (300, 3)).astype(np.float32)
    # adversarial points on and next to lattice planes, and the cube faces
    adv = []
    for N in TINY.resolutions:
        for k in range(N + 1):
            v = np.float32(k / N)
            for vv in (v, np.nextafter(v, np.float32(0)), np.nextafter(v, np.float32(1))):
                if 0 <= vv <= 1:
                    adv.append([vv, np.float32(0.3), np.float32(1.0)])
    pts = np.concatenate([pts, np.array(adv, np.float32)])
    _, idx, w = orc.encode(TINY, np.zeros(TINY.n_table_params, np.float32), pts, with_corners=True)
    for l, N in enumerate(TINY.resolutions):
        for i, x in enumerate(pts):
            c = [exact_cell(x[a], N) for a in range(3)]
            for e in range(8):
                v = [c[0] + (e & 1), c[1] + ((e >> 1) & 1), c[2] + ((e >> 2) & 1)]
                assert idx[l, i, e] == hash_index(v, N, T), (l, i, e)
            # trilinear weights: a partition of unity that reproduces x itself
            f = [Fraction(float(x[a])) * N - c[a] for a in range(3)]
            assert abs(w[l, i].sum() - 1.0) < 1e-15
            for a in range(3):
                bit = 1 << a
                pos = sum(w[l, i, e] * (c[a] + ((e & bit) > 0)) for e in range(8))
                assert abs(pos - float(Fraction(float(x[a])) * N)) < 1e-12
                assert 0 <= f[a] <= 1


def test_p8_dense_levels_are_a_bijection():
    arch = Arch(n_levels=2, log2_table=12, width=16, hidden=1, resolutions=(4, 15))  # 125, 4096
    for l, N in enumerate(arch.resolutions):
        g = (np.arange(N) + 0.5) / N
        z, y, x = np.meshgrid(g, g, g, indexing="ij")
        pts = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float32)
        _, idx, _ = orc.encode(arch, np.zeros(arch.n_table_params, np.float32), pts, with_corners=True)
        seen = np.unique(idx[l].ravel())
        np.testing.assert_array_equal(seen, np.arange((N + 1) ** 3))


def test_p9_encoding_constant_and_affine_tables():
    arch = Arch(n_levels=3, log2_table=12, width=16, hidden=1, resolutions=(3, 7, 15))  # all dense
    rng = np.random.default_rng(12)
    pts = rng.uniform(0, 1, (400, 3)).astype(np.float32)
    y = orc.encode(arch, np.full(arch.n_table_params, 0.75, np.float32), pts)
    np.testing.assert_allclose(y, 0.75, rtol=0, atol=1e-15)
    # affine table: entry of vertex v holds a . v / N + b (per feature)
    a = np.array([[0.5, -1.0, 2.0], [1.5, 0.25, -0.75]])
    b = np.array([0.125, -0.5])
    table = np.zeros((arch.n_levels, arch.table_size, 2))
    for l, N in enumerate(arch.resolutions):
        side = N + 1
        v = np.arange(side**3)
        vx, vy, vz = v % side, (v // side) % side, v // side**2
        X = np.stack([vx, vy, vz], 1) / N
        table[l, :side**3] = X @ a.T + b
    y = orc.encode(arch, table.astype(np.float32).ravel(), pts)
    for l in range(arch.n_levels):
        expect = pts.astype(np.float64) @ a.T + b
        np.testing.assert_allclose(y[l], expect, atol=2e-7)  # table rounded to FP32


# --------------------------------------------------------------------------
# P10: MLP reduces to matrix products

def test_p10_mlp_is_relu_matmul_chain():
    arch = Arch(n_levels=4, log2_table=10, width=32, hidden=3)
    rng = np.random.default_rng(13)
    mlp = init_params(arch, 3)[arch.n_table_params:]
    y = rng.normal(size=(50, arch.in_dim))
    Ws = [W.astype(np.float64) for W in mlp_layers(arch, mlp)]
    h = y.T
    for W in Ws[:-1]:
        h = np.maximum(W @ h, 0.0)
    expect = (Ws[-1] @ h).T
    np.testing.assert_allclose(orc.mlp_fwd(arch, mlp, y), expect, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------------
# P11: every gradient vs central finite differences of the oracle forward

def _fd_setup(loss_mode=0, lambda_d=0.3, lambda_sigma=1e-3, seed=14, n_rays=48):
    arch = Arch(n_levels=4, log2_table=8, width=16, hidden=2, base_res=4)
    rng = np.random.default_rng(seed)
    b = small_batch(3, seed=seed)
    pick = np.concatenate([np.nonzero(b.mask)[0][: n_rays // 2],
                           np.nonzero(b.mask == 0)[0][: n_rays // 2]])
    s = orc.sample(b.rays_o[pick], b.rays_d[pick], b.xi[pick][:, :16], n_coarse=0, n_fine=16,
                   include_coarse=False, uniform_only=True, eps=1e-4, near=NEAR, far=FAR,
                   world_to_obj=b.world_to_obj)
    params = init_params(arch, seed)
    params[:arch.n_table_params] = rng.uniform(-0.5, 0.5, arch.n_table_params)
    kw = dict(tgt_rgb=b.tgt_rgb[pick], tgt_depth=b.tgt_depth[pick], mask=b.mask[pick],
              bg=rng.uniform(0, 1, (len(pick), 3)).astype(np.float32),
              loss_mode=loss_mode, lambda_d=lambda_d, lambda_sigma=lambda_sigma)
    geo = (s["ray_obj"].astype(np.float32), s["t"].astype(np.float32),
           s["dt"].astype(np.float32), s["flags"])
    return arch, params, geo, kw, rng


@pytest.mark.parametrize("loss_mode", [0, 1])
def test_p11_gradients_match_central_differences(loss_mode):
    arch, params, geo, kw, rng = _fd_setup(loss_mode)
    g = orc.render_bwd(arch, params, *geo, **kw)

    def loss_and_sig(p):
        o = orc.render_fwd(arch, p, *geo, want_relu_signature=True, **kw)
        return o["loss"], o["relu_signature"]

    _, sig0 = loss_and_sig(params)
    nt = arch.n_table_params
    touched = np.nonzero(g[:nt])[0]
    coords = list(rng.choice(touched, size=min(64, touched.size), replace=False))
    coords += list(range(nt, arch.n_params))  # every MLP weight
    h = 1e-4
    gmax = np.abs(g).max()
    kinks = 0
    checked = 0
    for i in coords:
        pp, pm = params.copy(), params.copy()
        pp[i] = np.float32(params[i] + h)
        pm[i] = np.float32(params[i] - h)
        step = float(pp[i]) - float(pm[i])  # the exact step taken in FP32
        lp, sp = loss_and_sig(pp)
        lm, sm = loss_and_sig(pm)
        if not (np.array_equal(sp, sig0) and np.array_equal(sm, sig0)):
            kinks += 1
            continue
        fd = (lp - lm) / step
        checked += 1
        assert abs(fd - g[i]) <= 1e-4 * gmax + 1e-9, (i, fd, g[i])
    assert checked > 0.9 * len(coords), (checked, kinks)


def test_p11_prior_scene_full_architecture_central_differences():
    """The gradient check at the prior workload's architecture (16 levels x
    2^19, MLP 64 x 2) on its scene: colour MSE + 0.1 depth MSE with depth
    targets carrying 1 cm Gaussian noise; central differences of the FP64
    forward on 64 random touched hash entries and every one of the 6400 MLP
    weights, over 8 rays (4 meeting the object, 4 not).  The step is
    h = 1e-3; where a ReLU changes side within +-h (the loss has a kink
    there), h = 1e-4 and then 1e-5 are tried.  Parameters are perturbed in
    place, so no copy of the 16.8 M-entry array is made per coordinate."""
    from synth.arch import ARCH_LARGE
    from synth.workloads import LossSpec, prior_batch, prior_world
    arch = ARCH_LARGE
    w = prior_world(seed=1, pool_stride=9)
    b = prior_batch(w, 512, step=77, depth_noise=0.01, loss=LossSpec(lambda_d=0.1))
    pick = np.concatenate([np.nonzero(b.mask)[0][:4], np.nonzero(b.mask == 0)[0][:4]])
    s = b.sample
    r = orc.sample(b.rays_o[pick], b.rays_d[pick], b.xi[pick], n_coarse=s.n_coarse, n_fine=s.n_fine,
                   include_coarse=s.include_coarse, uniform_only=False, eps=s.eps, near=s.near, far=s.far,
                   world_to_obj=b.world_to_obj, prior=b.prior)
    geo = (r["ray_obj"].astype(np.float32), r["t"].astype(np.float32), r["dt"].astype(np.float32), r["flags"])
    params = init_params(arch, 3)
    rng = np.random.default_rng(15)
    params[:arch.n_table_params] = rng.uniform(-0.3, 0.3, arch.n_table_params).astype(np.float32)
    kw = dict(tgt_rgb=b.tgt_rgb[pick], tgt_depth=b.tgt_depth[pick], mask=b.mask[pick], lambda_d=np.float32(0.1))
    g = orc.render_bwd(arch, params, *geo, **kw)
    sig0 = orc.render_fwd(arch, params, *geo, want_relu_signature=True, **kw)["relu_signature"]
    nt = arch.n_table_params
    touched = np.nonzero(g[:nt])[0]
    coords = list(rng.choice(touched, size=64, replace=False)) + list(range(nt, arch.n_params))
    gmax = np.abs(g).max()

    def central(i, h):
        v = params[i]
        out = []
        for sgn in (1.0, -1.0):
            params[i] = np.float32(v + sgn * h)
            x = float(params[i])
            o = orc.render_fwd(arch, params, *geo, want_relu_signature=True, **kw)
            out.append((x, o["loss"], np.array_equal(o["relu_signature"], sig0)))
        params[i] = v
        (xp, lp, okp), (xm, lm, okm) = out
        return (lp - lm) / (xp - xm) if okp and okm else None

    checked, by_h = 0, {1e-3: 0, 1e-4: 0, 1e-5: 0}
    for i in coords:
        for h in (1e-3, 1e-4, 1e-5):
            fd = central(i, h)
            if fd is not None:
                assert abs(fd - g[i]) <= 1e-4 * gmax + 1e-9, (i, h, fd, g[i])
                checked += 1
                by_h[h] += 1
                break
    assert by_h[1e-3] > 0.3 * len(coords), by_h
    assert checked >= 0.95 * len(coords), (checked, by_h)


def test_p11_upstream_gradient_mode_is_vjp():
    """With upstream d_rgb / d_depth the backward is the vector-Jacobian
    product of (rgb, depth): compare with FD of sum(d_rgb*rgb + d_depth*depth)."""
    arch, params, geo, kw, rng = _fd_setup()
    n = geo[0].shape[0]
    d_rgb = rng.normal(size=(n, 3)).astype(np.float32)
    d_depth = rng.normal(size=n).astype(np.float32)
    g = orc.render_bwd(arch, params, *geo, bg=kw["bg"], d_rgb=d_rgb, d_depth=d_depth)

    def f(p):
        o = orc.render_fwd(arch, p, *geo, bg=kw["bg"])
        return (o["rgb"] * d_rgb).sum() + (o["depth"] * d_depth).sum()

    gmax = np.abs(g).max()
    for i in list(rng.choice(arch.n_params, 40, replace=False)) + [arch.n_params - 1]:
        pp, pm = params.copy(), params.copy()
        pp[i] = np.float32(params[i] + 1e-4)
        pm[i] = np.float32(params[i] - 1e-4)
        fd = (f(pp) - f(pm)) / (float(pp[i]) - float(pm[i]))
        assert abs(fd - g[i]) <= 2e-4 * gmax + 1e-9, (i, fd, g[i])


def _torch_render_loss(torch, arch, params, geo, kw, matmul, table_view):
    """The render + fused loss of the oracle's workload written in torch
    float64 autograd; `matmul(h, W)` forms each layer's product and
    `table_view(T)` what the forward gathers read of the tables.  Corner
    indices and weights (independent of the parameters) come from the
    oracle's encoder."""
    ray_obj, t, dt, flags = geo
    n, S = t.shape
    pos = orc.positions(ray_obj, t)  # FP32 positions as the kernels form them
    _, idx, w = orc.encode(arch, params[:arch.n_table_params], pos.reshape(-1, 3), with_corners=True)
    P = torch.tensor(params.astype(np.float64), requires_grad=True)
    T_ = arch.table_size
    tab = table_view(P[:arch.n_table_params]).view(arch.n_levels, T_, 2)
    ys = []
    for l in range(arch.n_levels):
        rows = tab[l][torch.tensor(idx[l].astype(np.int64))]          # [n*S, 8, 2]
        ys.append((rows * torch.tensor(w[l])[..., None]).sum(1))      # [n*S, 2]
    h = torch.cat(ys, 1)
    off = arch.n_table_params
    Ws = []
    for o_, i_ in arch.layer_shapes():
        Ws.append(P[off:off + o_ * i_].view(o_, i_))
        off += o_ * i_
    for W in Ws[:-1]:
        h = torch.relu(matmul(h, W))
    out = matmul(h, Ws[-1])
    sigma = torch.exp(out[:, 0]).view(n, S)
    col = torch.sigmoid(out[:, 1:]).view(n, S, 3)
    dtt = torch.tensor(dt.astype(np.float64))
    tt = torch.tensor(t.astype(np.float64))
    tau = sigma * dtt
    Tn = torch.exp(-torch.cat([torch.zeros(n, 1, dtype=torch.float64), torch.cumsum(tau, 1)[:, :-1]], 1))
    wgt = Tn * (1 - torch.exp(-tau))
    bg = torch.tensor(kw["bg"].astype(np.float64))
    C = (wgt[..., None] * col).sum(1) + torch.exp(-tau.sum(1))[:, None] * bg
    D = (wgt * tt).sum(1)
    live = torch.tensor((flags & orc.FLAG_MISS) == 0)
    C = torch.where(live[:, None], C, bg)
    D = torch.where(live, D, torch.zeros_like(D))
    m = torch.tensor(kw["mask"].astype(np.float64))
    tgt = torch.tensor(kw["tgt_rgb"].astype(np.float64))
    td = torch.tensor(kw["tgt_depth"].astype(np.float64))
    lam_d, lam_s = float(np.float32(kw["lambda_d"])), float(np.float32(kw["lambda_sigma"]))
    L = ((C - tgt) ** 2).sum() / (3 * n) + lam_d * (m * (D - td) ** 2).sum() / n \
        + lam_s * ((1 - m) * (sigma * live[:, None]).sum(1)).sum() / n
    L.backward()
    return L.item(), P.grad.numpy()


def test_p11_backward_matches_float64_autograd():
    """Independent cross-check of the hand-written adjoint: the same forward
    written with torch float64 autograd."""
    torch = pytest.importorskip("torch")
    arch, params, geo, kw, rng = _fd_setup(lambda_d=0.2, lambda_sigma=1e-2)
    g = orc.render_bwd(arch, params, *geo, **kw)
    L, gt = _torch_render_loss(torch, arch, params, geo, kw, lambda h, W: h @ W.T, lambda T: T)
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-12 * np.abs(g).max())
    lo = orc.render_fwd(arch, params, *geo, **kw)["loss"]
    assert abs(lo - L) < 1e-12


# --------------------------------------------------------------------------
# P15: reduced-precision emulation

def test_p15_rounding_matches_numpy_and_torch_casts():
    """The emulation's rounding (via FP32, nearest, ties to even) equals
    numpy's binary16 cast and torch's bfloat16 cast, over 12 decades plus
    subnormals, overflow and exact ties."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = rng.normal(size=200000) * np.exp(rng.uniform(-30, 12, 200000))
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11, 65504.0, 65519.0, 65520.0,
                     2.0 ** -24, 3 * 2.0 ** -25, 2.0 ** -25, -0.0, 0.0])
    x = np.concatenate([x, ties, -ties])
    with np.errstate(over="ignore"):
        ref16 = x.astype(np.float32).astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(orc.round16(x, "fp16"), ref16)
    refb = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.round16(x, "bf16"), refb)
    np.testing.assert_array_equal(orc.round16(x, "fp32"), x)


@pytest.mark.parametrize("mlp_dtype,table_dtype", [("bf16", "fp32"), ("fp16", "fp16")])
def test_p15_emulated_gradient_matches_rounded_autograd(mlp_dtype, table_dtype):
    """The emulated method against the same method written in torch float64
    autograd: each layer product takes operands rounded by torch's own casts
    (forward R(h) R(W)^T; adjoint R(g) R(W) and R(g)^T R(h)), the forward
    reads FP16-rounded table values with the gradient passed straight to the
    FP32 entries.  Both the loss and every gradient entry must agree."""
    torch = pytest.importorskip("torch")
    import dataclasses
    arch0, params, geo, kw, rng = _fd_setup(lambda_d=0.2, lambda_sigma=1e-2)
    arch = dataclasses.replace(arch0, mlp_dtype=mlp_dtype, table_dtype=table_dtype)
    tdt = {"bf16": torch.bfloat16, "fp16": torch.float16}[mlp_dtype]
    R = lambda x: x.to(torch.float32).to(tdt).to(torch.float64)

    class RoundedProduct(torch.autograd.Function):
        @staticmethod
        def forward(ctx, h, W):
            ctx.save_for_backward(h, W)
            return R(h) @ R(W).T

        @staticmethod
        def backward(ctx, g):
            h, W = ctx.saved_tensors
            return R(g) @ R(W), R(g).T @ R(h)

    def table_view(T):
        if table_dtype == "fp32":
            return T
        return T + (T.detach().to(torch.float32).to(torch.float16).to(torch.float64) - T.detach())

    L, gt = _torch_render_loss(torch, arch, params, geo, kw, RoundedProduct.apply, table_view)
    g = orc.render_bwd(arch, params, *geo, emulate=True, **kw)
    # with a loss scale the gradient operands are rounded scaled: round(g s) / s
    s_ = 4096.0
    Rs = lambda x: (x * s_).to(torch.float32).to(tdt).to(torch.float64) / s_

    class ScaledRoundedProduct(torch.autograd.Function):
        @staticmethod
        def forward(ctx, h, W):
            ctx.save_for_backward(h, W)
            return R(h) @ R(W).T

        @staticmethod
        def backward(ctx, g):
            h, W = ctx.saved_tensors
            return Rs(g) @ R(W), Rs(g).T @ R(h)

    _, gts = _torch_render_loss(torch, arch, params, geo, kw, ScaledRoundedProduct.apply, table_view)
    gs = orc.render_bwd(arch, params, *geo, emulate=True, loss_scale=s_, **kw)
    np.testing.assert_allclose(gs, gts, rtol=1e-9, atol=1e-12 * np.abs(gs).max())
    lo = orc.render_fwd(arch, params, *geo, emulate=True, **kw)["loss"]
    assert abs(lo - L) < 1e-12 * max(1.0, abs(L))
    np.testing.assert_allclose(g, gt, rtol=1e-9, atol=1e-12 * np.abs(g).max())
    # and it is not the plain method
    g_plain = orc.render_bwd(arch0, params, *geo, **kw)
    assert np.abs(g - g_plain).max() > 1e-6 * np.abs(g_plain).max()


# --------------------------------------------------------------------------
# P12: Adam

def test_p12_adam_matches_torch_float64():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(15)
    n = 1000
    p = rng.normal(size=n).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32) * 1e-3
    m = (rng.normal(size=n) * 1e-3).astype(np.float32)
    v = (rng.uniform(size=n) * 1e-6).astype(np.float32)
    lr, b1, b2, eps = 1e-2, 0.9, 0.99, 1e-15
    for step in (1, 7):
        P = torch.tensor(p.astype(np.float64), requires_grad=True)
        opt = torch.optim.Adam([P], lr=float(np.float32(lr)), betas=(float(np.float32(b1)),
                               float(np.float32(b2))), eps=float(np.float32(eps)))
        P.grad = torch.tensor(g.astype(np.float64))
        if step > 1:
            opt.state[P] = dict(step=torch.tensor(float(step - 1)),
                                exp_avg=torch.tensor(m.astype(np.float64)),
                                exp_avg_sq=torch.tensor(v.astype(np.float64)))
            mm, vv = m, v
        else:
            mm, vv = np.zeros(n, np.float32), np.zeros(n, np.float32)
        opt.step()
        po, mo, vo = orc.adam(p, g, mm, vv, lr=lr, beta1=b1, beta2=b2, eps=eps, step=step)
        np.testing.assert_allclose(po, P.detach().numpy(), rtol=1e-13, atol=1e-16)
        np.testing.assert_allclose(mo, opt.state[P]["exp_avg"].numpy(), rtol=1e-13)
        np.testing.assert_allclose(vo, opt.state[P]["exp_avg_sq"].numpy(), rtol=1e-13)


# --------------------------------------------------------------------------
# P13-P14: ground truth and losses

def test_p13_analytic_ground_truth_matches_riemann_sum():
    from synth.scene import riemann_ground_truth, sphere_box_scene
    b = small_batch(0)
    scene = sphere_box_scene()
    rng = np.random.default_rng(16)
    pick = np.concatenate([np.nonzero(b.mask)[0][:6], np.nonzero(b.mask == 0)[0][:2]])
    o, d = b.rays_o[pick].astype(np.float64), b.rays_d[pick].astype(np.float64)
    bg = rng.uniform(0, 1, 3)
    col, depth, hit, _ = scene.ground_truth(o, d, NEAR, FAR, bg=bg)
    ref = riemann_ground_truth(scene, o, d, NEAR, FAR, n_steps=200000, bg=bg)
    np.testing.assert_allclose(col, ref, atol=2e-4)


def test_p14_losses_closed_form():
    """Constant field (density e^2, colour 1/2): every colour, depth and
    density term is known in closed form, in both loss modes."""
    arch = Arch(n_levels=2, log2_table=8, width=16, hidden=1)
    p = const_model(arch, 2.0)
    rng = np.random.default_rng(17)
    n, S = 6, 5
    o, d = axis_rays(n, rng)
    ray_obj = np.concatenate([o + 0.5, d], 1).astype(np.float32)
    t = np.tile(np.float32([0.6, 0.8, 1.0, 1.2, 1.4]), (n, 1))
    dt = np.full((n, S), 0.25, np.float32)
    flags = np.zeros(n, np.uint8)
    flags[5] = orc.FLAG_MISS
    tgt = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    td = rng.uniform(0.5, 1.5, n).astype(np.float32)
    mask = np.array([1, 1, 1, 0, 0, 0], np.uint8)
    sig = math.exp(2.0)
    a = 1 - math.exp(-sig * 0.25)
    T = np.array([math.exp(-sig * 0.25 * j) for j in range(S)])
    w = T * a
    C = 0.5 * w.sum()
    D = float((w * t[0].astype(np.float64)).sum())
    Ch = np.array([[C] * 3] * 5 + [[0.0] * 3])
    Dh = np.array([D] * 5 + [0.0])
    for mode in (0, 1):
        lo = orc.render_fwd(arch, p, ray_obj, t, dt, flags, tgt_rgb=tgt, tgt_depth=td, mask=mask,
                            loss_mode=mode, lambda_d=0.5, lambda_sigma=0.1)
        e = Ch - tgt
        ed = Dh - td
        ssum = np.array([sig * S] * 5 + [0.0])
        ls = float(np.float32(0.1))  # the weights are handed over in FP32
        if mode == 0:
            L = (e**2).sum() / (3 * n) + 0.5 * (mask * ed**2).sum() / n + ls * ((1 - mask) * ssum).sum() / n
        else:
            L = np.sqrt((e**2).sum(1)).sum() + 0.5 * (mask * np.abs(ed)).sum() + ls * ((1 - mask) * ssum).sum()
        assert abs(lo["loss"] - L) < 1e-12 * max(1.0, abs(L)), (mode, lo["loss"], L)


# --------------------------------------------------------------------------
# the paper's printed constants

def test_paper_constants_fixture_matches_workload_defaults():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        g = json.load(f)
    from synth.workloads import PRIOR_SAMPLE, small_batch as sb
    assert sb(0).n_rays == g["rays_per_iteration"]["value"]
    assert PRIOR_SAMPLE.eps == g["epsilon"]["value"]
    from synth.prior import occupancy_prior  # noqa: F401  (R default)
    import inspect
    assert inspect.signature(occupancy_prior).parameters["R"].default == g["prior_grid_resolution"]["value"]
    assert g["n_coarse"]["value"] == g["n_fine"]["value"] == 32


# --------------------------------------------------------------------------
# P16: prior refresh (density grid of the NeRF, Sec. III-A "Normalized mesh
# generation"; recomputed every m iterations, Sec. III-B)

def refresh_params(arch, seed):
    """Parameters with a varied density field (table entries U(-0.3, 0.3))."""
    p = init_params(arch, seed)
    p[:arch.n_table_params] = np.random.default_rng(seed).uniform(-0.3, 0.3, arch.n_table_params).astype(np.float32)
    return p


def test_p16_refresh_of_constant_density_is_constant():
    """A model whose density is exp(s) everywhere refreshes to exp(s) at every vertex."""
    arch = ARCH_SMALL
    for s in (-2.0, 0.5, 3.0):
        grid = orc.prior_refresh(arch, const_model(arch, s), 9)
        np.testing.assert_allclose(grid, math.exp(s), rtol=1e-6)


def test_p16_refresh_equals_rendered_density_at_each_vertex():
    """Cross-path check: a one-sample ray placed exactly on vertex (i, j, k)
    (o = the vertex, t = 0) renders the density that the refreshed grid holds
    at [k][j][i] -- pins the vertex coordinates, the [z][y][x] layout and
    the split of the parameter vector."""
    arch = ARCH_SMALL
    R = 6
    p = refresh_params(arch, 3)
    grid = orc.prior_refresh(arch, p, R)
    idx = np.stack(np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij"), -1).reshape(-1, 3)  # (i, j, k)
    verts = (idx.astype(np.float64) / (R - 1)).astype(np.float32)
    n = verts.shape[0]
    ray_obj = np.concatenate([verts, np.tile(np.array([1.0, 0.0, 0.0], np.float32), (n, 1))], 1)
    t = np.zeros((n, 1), np.float32)
    dt = np.full((n, 1), 0.01, np.float32)
    out = orc.render_fwd(arch, p, ray_obj, t, dt, np.zeros(n, np.uint8), want_samples=True)
    sigma = out["samples"][:, 0, 0]
    np.testing.assert_allclose(grid[idx[:, 2], idx[:, 1], idx[:, 0]], sigma, rtol=1e-14)
    assert np.ptp(sigma) > 0.1 * np.abs(sigma).max()  # a varied field, so a transposed layout would fail


def test_p16_prior_lookup_reproduces_refreshed_grid_at_vertices():
    """The sampler's trilinear lookup (Eq. (4)) of a refreshed grid at its own
    vertices returns the stored values: refresh and lookup share one vertex
    alignment and one memory layout."""
    arch = ARCH_SMALL
    R = 7
    grid = orc.prior_refresh(arch, refresh_params(arch, 5), R)
    k, j, i = np.meshgrid(np.arange(R), np.arange(R), np.arange(R), indexing="ij")
    pts = np.stack([i, j, k], -1).reshape(-1, 3).astype(np.float64) / (R - 1)
    looked = orc.prior_lookup(grid.astype(np.float32), pts)
    np.testing.assert_allclose(looked, grid.astype(np.float32).reshape(-1).astype(np.float64), rtol=1e-12)


# P17: meta-learning (Sec. III-A, Eq. (1)-(2), Reptile)

def test_p17_sgd_equals_torch_sgd():
    """Eq. (1) against torch.optim.SGD (no momentum, no weight decay) in
    float64 over several steps with the same gradients."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(17)
    p0 = rng.normal(size=1000)
    lr = np.float32(0.37)
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SGD([w], lr=float(lr))
    p = p0.copy()
    for _ in range(4):
        g = rng.normal(size=1000)
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p = orc.sgd(p, g, lr=lr)
    np.testing.assert_allclose(p, w.detach().numpy(), rtol=0, atol=1e-15)


def test_p17_reptile_on_quadratic_tasks_matches_closed_form():
    """Tasks L_b(theta) = |theta - c_b|^2 / 2 (gradient theta - c_b).  q steps
    of Eq. (1) give c_b + (1 - eta)^q (theta - c_b), so Eq. (2) over B tasks
    gives theta + beta (1 - (1 - eta)^q) (mean_b c_b - theta): a wrong step
    count, sign, step size or mean fails it.  eta and beta are exact in FP32
    (the oracle takes them as the FP32 values the device receives)."""
    rng = np.random.default_rng(5)
    n = 64
    for B, q, eta, beta in ((1, 1, 0.5, 1.0), (1, 5, 0.25, 0.375), (4, 3, 0.125, 0.5), (7, 8, 0.0625, 0.75)):
        centres = rng.normal(size=(B, n))
        theta = rng.normal(size=n)
        grad = lambda c, k, p: p - c
        got = orc.reptile_meta_step(theta, list(centres), q=q, lr=eta, beta=beta, grad=grad, store=np.float64)
        want = theta + beta * (1.0 - (1.0 - eta) ** q) * (centres.mean(0) - theta)
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-13)


def test_p17_reptile_special_cases():
    """beta = 0 keeps theta; beta = 1 with one task is plain training of that
    task for q steps; tasks that return theta unchanged leave it unchanged."""
    rng = np.random.default_rng(8)
    theta = rng.normal(size=50)
    c = rng.normal(size=50)
    grad = lambda task, k, p: (p - task) * (1.0 + k)   # step-dependent, to pin the order of steps
    assert np.array_equal(orc.reptile_meta_step(theta, [c, -c], q=3, lr=0.125, beta=0.0, grad=grad,
                                                store=np.float64), theta)
    p = theta.copy()
    for k in range(3):
        p = p - 0.125 * grad(c, k, p)
    np.testing.assert_allclose(orc.reptile_meta_step(theta, [c], q=3, lr=0.125, beta=1.0, grad=grad,
                                                     store=np.float64), p, rtol=1e-15, atol=1e-15)
    np.testing.assert_array_equal(orc.reptile_outer(theta, [theta, theta], beta=0.7), theta)


# P18: canonical yaw (Sec. III-B, "Object State Canonicalization", Eq. (3))

def l_shape_points(rng, n):
    """Uniform points in an L-shaped solid with no yaw symmetry: the bar
    [-0.5, 0.5] x [-0.2, 0.2] x [-0.3, 0.3] plus the arm
    [0.2, 0.5] x [0.2, 0.5] x [-0.3, 0.3]."""
    out = []
    while sum(len(o) for o in out) < n:
        p = rng.uniform([-0.5, -0.2, -0.3], [0.5, 0.5, 0.3], (4 * n, 3))
        keep = (p[:, 1] <= 0.2) | (p[:, 0] >= 0.2)
        out.append(p[keep])
    return np.concatenate(out)[:n]


def l_shape_prior(R=32):
    """Occupancy of the L-shape on the vertices of its own extents box mapped
    onto the unit cube (u = (p - lo) / S), the normalisation Eq. (3) applies."""
    lo, hi = np.array([-0.5, -0.2, -0.3]), np.array([0.5, 0.5, 0.3])
    g = np.arange(R) / (R - 1)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    p = lo + np.stack([x, y, z], -1) * (hi - lo)
    occ = (p[..., 1] <= 0.2 + 1e-9) | (p[..., 0] >= 0.2 - 1e-9)
    return occ.astype(np.float32)


def rot_z(g):
    c, s = math.cos(g), math.sin(g)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


@pytest.mark.parametrize("k0", [0, 7, 29, 50])
def test_p18_recovers_a_known_yaw(k0):
    """The L-shape's cloud turned by -gamma_k0, moved and scaled: the search
    over K = 72 yaws returns k0 (rotating by gamma_k0 brings it back)."""
    rng = np.random.default_rng(k0)
    K = 72
    P = l_shape_points(rng, 4000) @ rot_z(-2 * math.pi * k0 / K).T
    P = (P * 1.7 + np.array([3.0, -2.0, 0.5])).astype(np.float32)
    r = orc.canonical_yaw(P, l_shape_prior(), K)
    assert r["best"] == k0
    s = np.sort(r["scores"])
    assert s[-1] > 1.01 * s[-2]            # a clear maximum (measured: 1.7% above the next)
    np.testing.assert_allclose(r["extents"][k0], [1.7, 1.19, 1.02], rtol=2e-3)


def test_p18_hand_worked_affine_prior():
    """F[k][j][i] = i, so F(u) = (R - 1) u_x exactly.  Points x = 0, 1, 3 on
    the x axis (y = z = 0: zero extents, normalised to 1/2).  gamma = 0:
    u_x = 0, 1/3, 1, score (R - 1) 4/3.  gamma = pi: x' = 0, -1, -3,
    u_x = 1, 2/3, 0, score (R - 1) 5/3.  K = 2, so the best index is 1."""
    R = 9
    F = np.broadcast_to(np.arange(R, dtype=np.float32), (R, R, R)).copy()
    P = np.array([[0, 0, 0], [1, 0, 0], [3, 0, 0]], np.float32)
    r = orc.canonical_yaw(P, F, 2)
    np.testing.assert_allclose(r["scores"], [(R - 1) * 4 / 3, (R - 1) * 5 / 3], rtol=1e-14)
    assert r["best"] == 1
    np.testing.assert_allclose(r["extents"][0], [3, 0, 0], atol=1e-15)
    np.testing.assert_allclose(r["centers"][0], [1.5, 0, 0], atol=1e-15)


def test_p18_invariances():
    """Scores do not change when the cloud is moved or scaled uniformly (by a
    power of two: exact in FP32); an exact quarter turn of the cloud shifts
    the score vector by K/4 indices; a constant prior c scores c |P| at every
    yaw."""
    rng = np.random.default_rng(4)
    K = 48
    P = rng.normal(size=(500, 3)).astype(np.float32) * np.float32([0.4, 0.2, 0.3])
    F = rng.uniform(0, 1, (17, 17, 17)).astype(np.float32)
    base = orc.canonical_yaw(P, F, K)["scores"]
    np.testing.assert_allclose(orc.canonical_yaw(P * np.float32(4), F, K)["scores"], base, rtol=1e-12)
    np.testing.assert_allclose(orc.canonical_yaw(P + np.float32([5, -3, 2]), F, K)["scores"], base, rtol=1e-6)
    quarter = np.stack([-P[:, 1], P[:, 0], P[:, 2]], 1)       # exact 90 degree turn
    # the turned cloud at gamma_k is the original at gamma_k + pi / 2
    np.testing.assert_allclose(orc.canonical_yaw(quarter, F, K)["scores"], np.roll(base, -(K // 4)), rtol=1e-12)
    const = orc.canonical_yaw(P, np.full((5, 5, 5), 0.75, np.float32), K)["scores"]
    np.testing.assert_allclose(const, 0.75 * len(P), rtol=1e-14)


def test_p18_degenerate_cloud_ties_to_first_yaw():
    """One repeated point: every extent is 0, every point normalises to the
    cube centre, all scores equal F(1/2, 1/2, 1/2) |P|, and the first yaw wins."""
    F = np.random.default_rng(2).uniform(0, 1, (5, 5, 5)).astype(np.float32)
    P = np.tile(np.float32([[0.3, -0.1, 0.2]]), (10, 1))
    r = orc.canonical_yaw(P, F, 16)
    centre = orc.prior_lookup(F, np.array([[0.5, 0.5, 0.5]]))[0]
    np.testing.assert_allclose(r["scores"], 10 * centre, rtol=1e-15)
    assert r["best"] == 0
    assert np.all(r["extents"] == 0)
