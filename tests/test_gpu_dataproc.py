"""The data processor and the image-combination steps on the GPU against the FP64 oracle:
SIN interpolation and deprojection grids of the 36-pointing mosaic geometry, beam
resampling, a plan built from the GPU grids, linear mosaicking and feathering."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dataproc as D

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2609_17636_amd import Plan  # noqa: E402
from paper_2609_17636_amd import dataproc as G  # noqa: E402

ARCSEC = np.pi / (180 * 3600)


def _mosaic_centres(n_sky, delta, ra0, dec0, rows_cols):
    """(ra, dec) of pointing centres given as sky-frame pixel positions (oracle projection)."""
    out = []
    for r, c in rows_cols:
        e = D.unproject((c - n_sky // 2) * delta, (r - n_sky // 2) * delta, ra0, dec0)
        out.append(D.radec(e))
    return np.array(out, dtype=np.float64)


@pytest.fixture(scope="module")
def geom():
    n_sky, n_sub, delta = 1024, 384, 30 * ARCSEC
    cen = synth.hex_centres(6, 6, 120.0, n_sky)
    radec = _mosaic_centres(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, cen)
    return n_sky, n_sub, delta, radec


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_sin_grids_match_the_oracle(geom, precision):
    n_sky, n_sub, delta, radec = geom
    got = G.sin_grids(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, radec, n_sub, delta, precision).double().cpu().numpy()
    worst = 0.0
    for k in (0, 7, 20, 35):
        want = D.sin_grid(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, n_sub, delta, *radec[k])
        worst = max(worst, float(np.abs(got[k] - want).max()))
    tol = 1e-7 if precision == "f64" else 2.5e-4  # f32: a few ulp of coordinates up to 1024
    print(f"[sin grids {precision}] max |d| {worst:.2e} px", flush=True)
    assert worst <= tol
    # the grids the synthetic mosaics are built from (an independent trigonometric form)
    g_syn, _ = synth.sin_interp(n_sky, n_sub, delta, synth.hex_centres(6, 6, 120.0, n_sky)[20])
    assert np.abs(got[20] - g_syn).max() <= tol


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_deprojection_grids_match_the_oracle(geom, precision):
    n_sky, n_sub, delta, radec = geom
    got = G.deprojection_grids(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, radec[:3], n_sub, delta,
                               precision).double().cpu().numpy()
    worst = 0.0
    for k in range(3):
        want, near = D.deprojection_grid(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, n_sub, delta, *radec[k])
        assert near.all()
        worst = max(worst, float(np.abs(got[k] - want).max()))
    print(f"[deprojection {precision}] max |d| {worst:.2e} px", flush=True)
    assert worst <= (1e-7 if precision == "f64" else 2.5e-4)


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_beam_resampling_matches_the_oracle(precision):
    rng = np.random.default_rng(70)
    nb, bd, n, d = 200, 45 * ARCSEC, 384, 30 * ARCSEC
    beams = rng.uniform(0, 1, (3, nb, nb))
    dt = torch.float32 if precision == "f32" else torch.float64
    got = G.resample_beams(torch.tensor(beams, dtype=dt, device="cuda"), bd, n, d).double().cpu().numpy()
    want = np.stack([D.resample_beam(b, bd, n, d) for b in beams])
    err = float(np.abs(got - want).max())
    print(f"[beam resampling {precision}] max |d| {err:.2e}", flush=True)
    # f32: coordinates up to nb are stored to ~nb * 2^-24 px, times a random beam's slope (<= 1 per px)
    assert err <= (1e-12 if precision == "f64" else 3e-5)


def test_plan_from_gpu_grids_and_beams():
    """The mini mosaic's objective with interpolation grids and beams made by the GPU data
    processor (a 2x beam image resampled to the sky pixel scale) against the oracle run on the
    same (oracle-made) grids and beams."""
    p = oracle.synthesize(synth.config_c3_mini())
    n_sky, n_sub, delta = p.n_sky, p.n_sub, p.pixel_rad
    cen = p.meta["centres"] if "centres" in p.meta else None
    assert cen is not None
    radec = _mosaic_centres(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, cen)
    fwhm = p.meta.get("fwhm_rad")
    nb = 2 * n_sub
    t = (np.arange(nb) - nb // 2) * (delta / 2)
    beam_img = np.exp(-4 * np.log(2) * (t[:, None] ** 2 + t[None, :] ** 2) / fwhm ** 2)
    beams_in = torch.tensor(np.repeat(beam_img[None], p.n_point, axis=0), dtype=torch.float32, device="cuda")
    q = p
    q.interp = G.sin_grids(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, radec, n_sub, delta).cpu().numpy()
    q.beams = G.resample_beams(beams_in, delta / 2, n_sub, delta).cpu().numpy()
    want_grid = np.stack([D.sin_grid(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, n_sub, delta, *rd) for rd in radec])
    want_beams = np.stack([D.resample_beam(beam_img, delta / 2, n_sub, delta)] * p.n_point)
    assert np.abs(q.interp - want_grid).max() <= 2.5e-4 and np.abs(q.beams - want_beams).max() <= 2e-6
    plan = Plan.from_problem(q)
    plan.set_problem_data(q)
    x = np.random.default_rng(71).uniform(0, 50, size=q.x_true.shape)
    terms, grad = plan.objective_grad(torch.tensor(x, dtype=torch.float32, device="cuda"))
    q.interp, q.beams = want_grid, want_beams.astype(np.float32)
    want_t, want_g = oracle.objective_grad(q, x)
    rq = abs(terms[0] - want_t["Q_tot"]) / want_t["Q_tot"]
    rg = np.linalg.norm(grad.double().cpu().numpy() - want_g) / np.linalg.norm(want_g)
    print(f"[plan from GPU grids] relQ {rq:.2e} relG {rg:.2e}", flush=True)
    assert rq <= 1e-5 and rg <= 1e-5


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_linear_mosaic_matches_the_oracle(precision):
    rng = np.random.default_rng(72)
    n_sky, n_sub, delta = 256, 96, 30 * ARCSEC
    cen = synth.hex_centres(2, 3, 60.0, n_sky)
    radec = _mosaic_centres(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, cen)
    P, C = len(radec), 3
    subs = rng.uniform(0, 5, (P, C, n_sub, n_sub))
    beams = np.stack([synth.gaussian_pb(n_sub, delta, 40 * delta)] * P)
    dt = torch.float32 if precision == "f32" else torch.float64
    dep = G.deprojection_grids(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, radec, n_sub, delta, precision)
    img, peff = G.linear_mosaic(torch.tensor(subs, dtype=dt, device="cuda"), torch.tensor(beams, dtype=dt, device="cuda"),
                                dep, pb_min=0.2)
    want_dep = np.stack([D.deprojection_grid(n_sky, delta, synth.LMC_RA, synth.LMC_DEC, n_sub, delta, *rd)[0]
                         for rd in radec])
    want_img, want_peff = D.linear_mosaic(subs, beams, want_dep, pb_min=0.2)
    got, gp = img.double().cpu().numpy(), peff.double().cpu().numpy()
    e1 = np.linalg.norm(got - want_img) / np.linalg.norm(want_img)
    e2 = float(np.abs(gp - want_peff).max())
    print(f"[linear mosaic {precision}] rel {e1:.2e} pb_eff {e2:.2e}", flush=True)
    assert e1 <= (1e-10 if precision == "f64" else 1e-5) and e2 <= (1e-12 if precision == "f64" else 1e-5)


@pytest.mark.parametrize("precision,n", [("f32", 1024), ("f64", 256), ("f32", 64)])
def test_feather_matches_the_oracle(precision, n):
    rng = np.random.default_rng(73)
    C, delta, theta = 2, 30 * ARCSEC, 30 * 60 * ARCSEC
    interf = rng.standard_normal((C, n, n))
    sd = synth.lognormal_field(synth.grf_k3(rng, n))[None].repeat(C, axis=0) * 0.1
    dt = torch.float32 if precision == "f32" else torch.float64
    got = G.feather(torch.tensor(interf, dtype=dt, device="cuda"), torch.tensor(sd, dtype=dt, device="cuda"),
                    delta, theta).double().cpu().numpy()
    want = D.feather(interf, sd, delta, theta)
    e = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"[feather {precision} n={n}] rel {e:.2e}", flush=True)
    assert e <= (1e-10 if precision == "f64" else 1e-5)
