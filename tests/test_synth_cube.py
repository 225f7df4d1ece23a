"""The shared-uv cube generator: layout, per-channel scales and flux scales, and blocks
that do not depend on how many threads fill them."""
import numpy as np

import synth


def test_cube_layout_and_channel_scales():
    p = synth.config_c4_mini()
    P, C = p.n_point, p.n_chan
    mk = np.diff(p.pt_offsets)
    assert p.vis_offsets.size == P * C + 1
    assert np.array_equal(np.diff(p.vis_offsets), np.repeat(mk, C))
    assert p.uv.shape == (p.pt_offsets[-1], 2) and p.weight.shape == (p.pt_offsets[-1],)
    f = p.meta["freqs"]
    assert np.allclose(np.diff(f), 25e6) and np.isclose(f.mean(), 1.4e9)
    assert np.allclose(p.uv_scale, f / 1.4e9)
    # Rayleigh-Jeans flux scale grows as nu^2
    assert np.allclose(p.flux_scale / p.flux_scale[0], (f / f[0]) ** 2)
    # channel c of pointing k sees the pointing's track times nu_c / nu_ref
    k, c = 1, 2
    s = slice(int(p.pt_offsets[k]), int(p.pt_offsets[k + 1]))
    assert np.array_equal(p.uv_of(k, c), p.uv[s].astype(np.float64) * p.uv_scale[c])
    # flag rate of each block below its cap, noise unit variance per component
    for b in range(P * C):
        fl = p.flags[p.vis_offsets[b]:p.vis_offsets[b + 1]]
        assert fl.mean() <= 0.3 + 0.05
    v = p.vis.view(np.float32)
    assert abs(v.std() - 1.0) < 0.01


def test_cube_blocks_do_not_depend_on_thread_count():
    a = synth.cube("t", 7, 64, 30.0, 2, 2, 16.0, 16.0, 32, 10, 3, 0.2, 1.4e9, 1e6, sd_n=8,
                   sd_fwhm_arcmin=4.0, with_field=False, threads=1)
    b = synth.cube("t", 7, 64, 30.0, 2, 2, 16.0, 16.0, 32, 10, 3, 0.2, 1.4e9, 1e6, sd_n=8,
                   sd_fwhm_arcmin=4.0, with_field=False, threads=5)
    assert np.array_equal(a.flags, b.flags)
    assert np.array_equal(a.vis, b.vis)
    assert np.array_equal(a.uv, b.uv)


def test_expand_writes_the_cube_out_per_block():
    p = synth.config_c4_mini()
    e = p.expand()
    assert e.n_vis == p.n_vis
    for k in range(p.n_point):
        for c in range(p.n_chan):
            s = p.block(k, c)
            assert np.array_equal(e.uv[s], p.uv_of(k, c))
            assert np.array_equal(e.weight[s], p.weight_of(k))
