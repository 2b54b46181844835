"""GPU parity of the spherical harmonic transforms against the oracle."""
import math
import sys

import numpy as np
import pytest

from oracle import geometry, sht
from oracle.legendre import LegendreSweep

pytestmark = pytest.mark.gpu

SHT_TOL = 1e-10  # relative (max-abs error over max-abs value), per SHT


def _setup():
    import torch
    from paper_1710_00621_amd import crsolve
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch, crsolve


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


CASES = [
    (("gl", 33, 65), 32, 1),
    (("gl", 6, 7), 9, 2),        # nphi < 2L+1: aliasing on every ring
    (("healpix", 1), 3, 1),
    (("healpix", 8), 16, 3),
    (("healpix", 16), 40, 2),    # L > 2 Nside: polar rings alias
    (("healpix", 32), 70, 1),    # ragged: 127 rings, 64 pairs, odd L
    (("healpix", 64), 128, 9),   # several ring tiles, nmaps > 8
    (("healpix", 13), 0, 1),     # lmax = 0, odd Nside (non power-of-two rings)
    (("healpix", 37), 90, 2),    # cap rings 4i with prime i: Bluestein lengths
    (("gl", 5, 4093), 40, 1),    # odd prime ring length above 2048: full-length Bluestein
    (("gl", 9, 1), 4, 1),        # one pixel per ring: everything aliases onto m = 0
    (("gl", 7, 2046), 1100, 1),  # even length 2 * 3 * 11 * 31: half-length Bluestein
    (("gl", 5, 4375), 40, 1),    # odd 5^4 * 7 above 4096: full-length direct FFT, longest tier
    (("gl", 3, 8190), 30, 2),    # 8190 = 2 * 4095 (factor 13): Bluestein of 8192 points
    (("healpix", 37), 90, 5),    # Bluestein caps, five maps
    (("gl", 6, 7), 9, 4),        # odd aliasing rings, four maps
]


@pytest.mark.parametrize("spec,lmax,nmaps", CASES)
def test_sht_synth_and_adjoint_match_oracle(spec, lmax, nmaps):
    torch, crsolve = _setup()
    print(f"case synth/adjoint {spec} lmax={lmax} nmaps={nmaps}", flush=True)
    g = crsolve.Grid.from_spec(spec)
    og = geometry.make_grid(spec)
    assert g.npix == og.npix
    rng = np.random.default_rng(7)
    alm = rng.standard_normal((nmaps, sht.nalm(lmax)))
    maps = rng.standard_normal((nmaps, og.npix))
    ref_map = sht.synth(og, lmax, alm)
    ref_alm = sht.adjoint(og, lmax, maps)
    dev = torch.device("cuda")
    got_map = crsolve.sht_synth(g, lmax, torch.tensor(alm, device=dev)).cpu().numpy()
    got_alm = crsolve.sht_adjoint(g, lmax, torch.tensor(maps, device=dev)).cpu().numpy()
    assert _rel(got_map, ref_map) < SHT_TOL
    assert _rel(got_alm, ref_alm) < SHT_TOL


def test_grid_geometry_matches_oracle():
    torch, crsolve = _setup()
    for spec in (("healpix", 1), ("healpix", 5), ("healpix", 64), ("gl", 33, 65), ("gl", 17, 40)):
        g = crsolve.Grid.from_spec(spec)
        og = geometry.make_grid(spec)
        z, phi = g.pixel_centres()
        oz, ophi = og.pixel_centres()
        np.testing.assert_allclose(z, oz, atol=2e-16)
        np.testing.assert_allclose(phi, ophi, atol=1e-14)
        np.testing.assert_allclose(g.weights(), og.pixel_weights(), rtol=1e-12)


def test_gl_round_trip_on_device():
    """Y^T W Y = I on the 33 x 65 GL grid at L = 32 (Sect. 2.1).  The bound
    allows O(10 eps L log2 M) for two Legendre sums over 33 rings and two
    ring FFTs of length 65 = 5 * 13, which run as length-256 Bluestein
    convolutions."""
    torch, crsolve = _setup()
    g = crsolve.Grid.gauss_legendre(33, 65)
    w = torch.tensor(g.weights(), device="cuda")
    a = torch.randn(4, sht.nalm(32), dtype=torch.float64, device="cuda")
    back = crsolve.sht_adjoint(g, 32, crsolve.sht_synth(g, 32, a) * w)
    assert float((back - a).abs().max()) < 5e-13


def test_adjoint_identity_and_determinism():
    torch, crsolve = _setup()
    g = crsolve.Grid.healpix(32)
    L = 96
    gen = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randn(2, sht.nalm(L), dtype=torch.float64, device="cuda", generator=gen)
    y = torch.randn(2, g.npix, dtype=torch.float64, device="cuda", generator=gen)
    yx = crsolve.sht_synth(g, L, x)
    xty = crsolve.sht_adjoint(g, L, y)
    lhs = (yx * y).sum(dim=1)
    rhs = (x * xty).sum(dim=1)
    # rounding error of <Yx, y> - <x, Y^T y> scales with |Yx| |y| (the dot
    # products themselves can be small by cancellation)
    scale = yx.norm(dim=1) * y.norm(dim=1)
    assert float(((lhs - rhs).abs() / scale).max()) < 1e-13
    # bitwise determinism (fixed-order reductions)
    assert torch.equal(crsolve.sht_adjoint(g, L, y), xty)
    assert torch.equal(crsolve.sht_synth(g, L, x), yx)


def _ring_subset(og, rings):
    """Oracle grid restricted to some rings (for sampled checks at full size)."""
    sub = geometry.Grid(og.kind, og.z[rings], og.sint[rings], og.nphi[rings], og.phi0[rings],
                        og.ring_weight[rings], og.params)
    return sub


@pytest.mark.parametrize("nside,lmax", [(256, 512), (1024, 2000)])
def test_sht_full_size_sampled(nside, lmax):
    """At the large band shapes: synthesis checked on sampled rings (polar,
    cap/belt boundary, equator) and the adjoint on sampled m, each computed
    by the oracle one ring / one m at a time."""
    torch, crsolve = _setup()
    print(f"case full-size sampled nside={nside} lmax={lmax}", flush=True)
    g = crsolve.Grid.healpix(nside)
    og = geometry.healpix(nside)
    rng = np.random.default_rng(11)
    nal = sht.nalm(lmax)
    ell = sht.lm_arrays(lmax)[0]
    alm = rng.standard_normal(nal) / np.sqrt(1.0 + ell)  # red spectrum, like the sky
    dev = torch.device("cuda")
    got = crsolve.sht_synth(g, lmax, torch.tensor(alm, device=dev)).cpu().numpy()
    rings = [0, 1, 7, nside - 2, nside - 1, 2 * nside - 1, 3 * nside + 5, og.nring - 1]
    sub = _ring_subset(og, np.array(rings))
    ref = sht.synth(sub, lmax, alm)
    gs = np.concatenate([got[og.offset[r]:og.offset[r] + og.nphi[r]] for r in rings])
    assert _rel(gs, ref) < SHT_TOL
    # adjoint: sampled m, full ring sum in the oracle
    maps = rng.standard_normal(og.npix)
    got_a = crsolve.sht_adjoint(g, lmax, torch.tensor(maps, device=dev)).cpu().numpy()
    ms = [0, 1, 2, lmax // 3, lmax - 1, lmax]
    Hc = np.zeros((og.nring, lmax + 1))
    Hs = np.zeros((og.nring, lmax + 1))
    for r in range(og.nring):
        phi = og.ring_phi(r)
        f = maps[og.offset[r]:og.offset[r] + og.nphi[r]]
        arg = np.outer(phi, ms)
        Hc[r, ms] = f @ np.cos(arg)
        Hs[r, ms] = f @ np.sin(arg)
    sweep = LegendreSweep(og.z, og.sint, lmax)
    for m in ms:
        sweep.skip_to(m)
        lam = sweep.table(m)
        n = lmax - m + 1
        o = sht.m_offset(lmax, m)
        c = 1.0 if m == 0 else math.sqrt(2.0)
        refc = c * (Hc[:, m] @ lam)
        assert _rel(got_a[o:o + n], refc) < SHT_TOL, m
        if m > 0:
            refs = c * (Hs[:, m] @ lam)
            assert _rel(got_a[o + n:o + 2 * n], refs) < SHT_TOL, m


def _sampled_adjoint_ref(og, lmax, maps, ms):
    """Oracle adjoint coefficients at the sampled m for every map (rows)."""
    nm = maps.shape[0]
    Hc = np.zeros((nm, og.nring, len(ms)))
    Hs = np.zeros((nm, og.nring, len(ms)))
    for r in range(og.nring):
        phi = og.ring_phi(r)
        f = maps[:, og.offset[r]:og.offset[r] + og.nphi[r]]
        arg = np.outer(phi, ms)
        Hc[:, r] = f @ np.cos(arg)
        Hs[:, r] = f @ np.sin(arg)
    sweep = LegendreSweep(og.z, og.sint, lmax)
    out = {}
    for i, m in enumerate(ms):
        sweep.skip_to(m)
        lam = sweep.table(m)
        c = 1.0 if m == 0 else math.sqrt(2.0)
        out[m] = (c * (Hc[:, :, i] @ lam), c * (Hs[:, :, i] @ lam))
    return out


def test_sht_full_size_sampled_many_maps():
    """Nside 1024, L = 2000 with 6 maps (the matrix-core kernels at the size
    and launch configuration of the benchmark): synthesis on sampled rings
    and the adjoint on sampled m for every map, against the oracle."""
    torch, crsolve = _setup()
    nside, lmax, nm = 1024, 2000, 6
    print(f"case full-size sampled nside={nside} lmax={lmax} nmaps={nm}", flush=True)
    g = crsolve.Grid.healpix(nside)
    og = geometry.healpix(nside)
    rng = np.random.default_rng(12)
    ell = sht.lm_arrays(lmax)[0]
    alm = rng.standard_normal((nm, sht.nalm(lmax))) / np.sqrt(1.0 + ell)
    dev = torch.device("cuda")
    got = crsolve.sht_synth(g, lmax, torch.tensor(alm, device=dev)).cpu().numpy()
    rings = [0, 3, nside - 1, 2 * nside - 1, 3 * nside + 5, og.nring - 2]
    sub = _ring_subset(og, np.array(rings))
    ref = sht.synth(sub, lmax, alm)
    gs = np.concatenate([got[:, og.offset[r]:og.offset[r] + og.nphi[r]] for r in rings], axis=1)
    assert _rel(gs, ref) < SHT_TOL
    maps = rng.standard_normal((nm, og.npix))
    got_a = crsolve.sht_adjoint(g, lmax, torch.tensor(maps, device=dev)).cpu().numpy()
    ms = [0, 1, 5, 700, lmax - 2, lmax]
    ref_a = _sampled_adjoint_ref(og, lmax, maps, ms)
    for m in ms:
        n = lmax - m + 1
        o = sht.m_offset(lmax, m)
        assert _rel(got_a[:, o:o + n], ref_a[m][0]) < SHT_TOL, m
        if m > 0:
            assert _rel(got_a[:, o + n:o + 2 * n], ref_a[m][1]) < SHT_TOL, m


FORCED = [
    # (environment, nmaps): every kernel variant the launchers choose between,
    # forced at a size the oracle checks in full (ragged tiles: 80 ring pairs)
    ({"CRS_LEG_RS": "1", "CRS_LEG_RA": "1"}, 1),
    ({"CRS_LEG_RS": "2", "CRS_LEG_RA": "2"}, 1),
    ({"CRS_LEG_RS": "4", "CRS_LEG_RA": "4"}, 1),
    ({"CRS_LEG_RS": "2", "CRS_LEG_RA": "4"}, 2),
    ({"CRS_LEG_RA": "2"}, 3),
    ({"CRS_LEG_TA": "1"}, 9),
    ({"CRS_LEG_TA": "2"}, 9),
    ({"CRS_LEG_TA": "2", "CRS_LEG_MFMA_MIN": "1"}, 1),
]


@pytest.mark.parametrize("env,nmaps", FORCED)
def test_sht_kernel_variants_match_oracle(env, nmaps, monkeypatch):
    torch, crsolve = _setup()
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    print(f"case variants {env} nmaps={nmaps}", flush=True)
    spec, lmax = ("healpix", 40), 90
    g = crsolve.Grid.from_spec(spec)
    og = geometry.make_grid(spec)
    rng = np.random.default_rng(21)
    alm = rng.standard_normal((nmaps, sht.nalm(lmax)))
    maps = rng.standard_normal((nmaps, og.npix))
    dev = torch.device("cuda")
    got_map = crsolve.sht_synth(g, lmax, torch.tensor(alm, device=dev)).cpu().numpy()
    got_alm = crsolve.sht_adjoint(g, lmax, torch.tensor(maps, device=dev)).cpu().numpy()
    assert _rel(got_map, sht.synth(og, lmax, alm)) < SHT_TOL
    assert _rel(got_alm, sht.adjoint(og, lmax, maps)) < SHT_TOL


def test_autotuned_legendre_matches_oracle():
    """The autotuner records one of the variants for the shape; transforms of
    that shape then use it and still match the oracle."""
    torch, crsolve = _setup()
    spec, lmax, nmaps = ("healpix", 24), 60, 5
    print(f"case autotune {spec} lmax={lmax} nmaps={nmaps}", flush=True)
    g = crsolve.Grid.from_spec(spec)
    og = geometry.make_grid(spec)
    c = crsolve.autotune_legendre(g, lmax, nmaps)
    assert c == crsolve.legendre_choice(g, lmax, nmaps)
    assert c["synth_mfma"] in (0, 1) and c["adjoint_mfma"] in (0, 1)
    assert c["synth_pairs_per_lane"] in (1, 2, 4) and c["adjoint_pairs_per_lane"] in (1, 2, 4)
    assert c["adjoint_tiles_per_wave"] in (1, 2)
    rng = np.random.default_rng(23)
    alm = rng.standard_normal((nmaps, sht.nalm(lmax)))
    maps = rng.standard_normal((nmaps, og.npix))
    dev = torch.device("cuda")
    got_map = crsolve.sht_synth(g, lmax, torch.tensor(alm, device=dev)).cpu().numpy()
    got_alm = crsolve.sht_adjoint(g, lmax, torch.tensor(maps, device=dev)).cpu().numpy()
    assert _rel(got_map, sht.synth(og, lmax, alm)) < SHT_TOL
    assert _rel(got_alm, sht.adjoint(og, lmax, maps)) < SHT_TOL


def test_ring_launch_classes_agree(monkeypatch):
    """Nside 512, L = 1024: with 8 maps every ring class of the long tier
    (Bluestein caps) runs on its own power-of-two kernel; with one map the
    classes too small to fill the GPU are merged into one launch of the
    general kernel.  Both launch plans must give the same transforms (the
    Legendre stage is held to the same vector kernels, so only the ring
    stage's launch plan differs; short rings fold with another block size)."""
    torch, crsolve = _setup()
    monkeypatch.setenv("CRS_LEG_MFMA_MIN", "100")
    nside, lmax, nm = 512, 1024, 8
    print(f"case ring classes nside={nside} lmax={lmax} nmaps={nm} vs 1", flush=True)
    g = crsolve.Grid.healpix(nside)
    dev = torch.device("cuda")
    gen = torch.Generator(device="cpu").manual_seed(31)
    alm = torch.randn(nm, (lmax + 1) ** 2, generator=gen, dtype=torch.float64).to(dev)
    maps = torch.randn(nm, g.npix, generator=gen, dtype=torch.float64).to(dev)
    many_map = crsolve.sht_synth(g, lmax, alm).cpu().numpy()
    many_alm = crsolve.sht_adjoint(g, lmax, maps).cpu().numpy()
    for j in range(nm):
        one_map = crsolve.sht_synth(g, lmax, alm[j:j + 1]).cpu().numpy()
        one_alm = crsolve.sht_adjoint(g, lmax, maps[j:j + 1]).cpu().numpy()
        assert _rel(one_map[0], many_map[j]) < 1e-13, j
        assert _rel(one_alm[0], many_alm[j]) < 1e-13, j


def test_gl_round_trip_large():
    """Y^T W Y = I at L = 4000 on the 4001 x 8192 Gauss-Legendre grid (exact
    quadrature: 4001 nodes integrate degree 2L, 8192 >= 2L + 1 points per
    ring): rings of 8192 pixels, the recurrence deep into underflow at high
    m.  Two transforms, so twice the per-transform bound."""
    torch, crsolve = _setup()
    nring, nphi, lmax = 4001, 8192, 4000
    print(f"case GL round trip {nring}x{nphi} lmax={lmax}", flush=True)
    g = crsolve.Grid.gauss_legendre(nring, nphi)
    w = torch.tensor(g.weights(), device="cuda")
    gen = torch.Generator(device="cpu").manual_seed(41)
    a = torch.randn(1, sht.nalm(lmax), generator=gen, dtype=torch.float64).to("cuda")
    back = crsolve.sht_adjoint(g, lmax, crsolve.sht_synth(g, lmax, a) * w)
    err = float((back - a).abs().max() / a.abs().max())
    print(f"round trip max rel error {err:.3e}", flush=True)
    assert err < 2 * SHT_TOL


def test_sht_nside2048_l6000_sampled():
    """Full resolution (Nside 2048: 8192-pixel rings, L = 6000): the adjoint
    on sampled m for every ring against the oracle, and the synthesis tied to
    it by the adjoint identity <Y x, y> = <x, Y^T y>."""
    torch, crsolve = _setup()
    nside, lmax = 2048, 6000
    print(f"case full resolution nside={nside} lmax={lmax}", flush=True)
    g = crsolve.Grid.healpix(nside)
    og = geometry.healpix(nside)
    rng = np.random.default_rng(43)
    maps = rng.standard_normal((1, og.npix))
    dev = torch.device("cuda")
    y = torch.tensor(maps, device=dev)
    got_a = crsolve.sht_adjoint(g, lmax, y)
    ms = [0, 1, 3000, lmax - 1, lmax]
    ref_a = _sampled_adjoint_ref(og, lmax, maps, ms)
    ga = got_a.cpu().numpy()
    for m in ms:
        n = lmax - m + 1
        o = sht.m_offset(lmax, m)
        assert _rel(ga[:, o:o + n], ref_a[m][0]) < SHT_TOL, m
        if m > 0:
            assert _rel(ga[:, o + n:o + 2 * n], ref_a[m][1]) < SHT_TOL, m
    ell = sht.lm_arrays(lmax)[0]
    x = torch.tensor(rng.standard_normal((1, sht.nalm(lmax))) / np.sqrt(1.0 + ell), device=dev)
    yx = crsolve.sht_synth(g, lmax, x)
    lhs = float((yx * y).sum())
    rhs = float((x * got_a).sum())
    assert abs(lhs - rhs) / float(yx.norm() * y.norm()) < 1e-13


def test_reserve_then_transforms_allocate_nothing():
    """crs_sht_reserve builds the tables and the workspace up front: the
    transforms that follow (up to the reserved map count) leave the device's
    free memory unchanged and match the transforms of another grid object."""
    torch, crsolve = _setup()
    print("case reserve: healpix 64, lmax 128, 5 maps", flush=True)
    lmax, nm = 128, 5
    gen = torch.Generator(device="cpu").manual_seed(41)
    g2 = crsolve.Grid.healpix(64)
    alm = torch.randn(nm, (lmax + 1) ** 2, generator=gen, dtype=torch.float64).cuda()
    maps = torch.randn(nm, g2.npix, generator=gen, dtype=torch.float64).cuda()
    out_map = torch.empty(nm, g2.npix, dtype=torch.float64, device="cuda")
    out_alm = torch.empty(nm, (lmax + 1) ** 2, dtype=torch.float64, device="cuda")
    # reference on a grid of its own (also warms torch's allocator for these shapes)
    ref_map = crsolve.sht_synth(g2, lmax, alm[:2]).cpu().numpy()
    ref_alm = crsolve.sht_adjoint(g2, lmax, maps[:2]).cpu().numpy()
    g = crsolve.Grid.healpix(64)
    g.reserve(lmax, nm)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for k in (nm, 2):
        crsolve.sht_synth(g, lmax, alm[:k], out=out_map[:k])
        crsolve.sht_adjoint(g, lmax, maps[:k], out=out_alm[:k])
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert _rel(out_map[:2].cpu().numpy(), ref_map) < 1e-13
    assert _rel(out_alm[:2].cpu().numpy(), ref_alm) < 1e-13
