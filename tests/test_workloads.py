"""The seeded synthetic inputs (workloads/) have the shapes, ranges and
structure their recipes state: the uneven batch's sizes, aspect ratios,
frequencies and spacing; the 128^3 layered model's layers and perturbation;
the 96^3 FWI model's sphere and smoothed start; the 320x320x160 model's body,
smoothing and acquisition.  Each generator is deterministic (seeded)."""
import numpy as np
from scipy import ndimage

import workloads as W


def test_uneven_batch_recipe():
    ps = W.c4_problem_params(count=256)
    assert len(ps) == 256 and ps == W.c4_problem_params(count=256)
    for p in ps:
        n = np.array(p["n"])
        assert n.min() >= 48 and n.max() <= 160 and n.max() <= 2 * n.min()
        assert 3.0 <= p["freq"] <= 12.0 and p["npml"] == 8
        assert abs(p["h"] - 1500.0 / (8.0 * p["freq"])) <= 1e-12 * p["h"]
    # the draw's total size, as the benchmark reports it
    assert sum(int(np.prod(p["n"])) for p in ps) == 324608331
    w = W.c4_problem(ps[0])
    si = W.interior_shape(w.n, w.npml)
    v = w.v[w.npml:-w.npml, w.npml:-w.npml, w.npml:-w.npml]
    assert v.shape == si and v.min() == 1500.0 and v.max() == 4500.0
    assert np.array_equal(w.v[0], w.v[w.npml])  # layer = nearest interior value
    assert w.src.tolist() == [[w.n[0] // 2, w.n[1] // 2, w.npml + 2]]


def test_layered_128cube_recipe():
    w = W.c2_layered()
    assert w.n == (128, 128, 128) and w.h == 12.5 and w.npml == 15 and w.freq == 8.0
    si = W.interior_shape(w.n, w.npml)
    vb = W.layered_velocity(si, 6, 1500.0, 4500.0, 2.0)
    v = w.v[15:-15, 15:-15, 15:-15]
    xi = (v / vb - 1.0) / 0.05  # the perturbation field: zero mean, unit std
    assert abs(xi.mean()) <= 1e-10 and abs(xi.std() - 1.0) <= 1e-10
    prof = vb[0, 0]
    assert np.all(np.diff(prof) >= 0.0) and abs(prof[0] - 1500.0) < 1.0 and abs(prof[-1] - 4500.0) < 1.0
    # 16 sources on a 4 x 4 array on the first interior plane, cell-centred
    xs = 15 + np.floor((np.arange(4) + 0.5) * 98 / 4).astype(int)
    assert sorted(map(tuple, w.src.tolist())) == sorted((a, b, 15) for a in xs for b in xs)
    assert np.array_equal(W.c2_layered().v, w.v)


def test_fwi_96cube_recipe():
    w = W.c3_fwi()
    assert w.n == (96, 96, 96) and w.h == 30.0 and w.npml == 10 and w.freq == 5.0
    si = W.interior_shape(w.n, w.npml)
    vb = W.layered_velocity(si, 6, 1500.0, 4500.0, 2.0)
    vt = w.v_true[10:-10, 10:-10, 10:-10]
    inside = np.isclose(vt, 0.85 * vb, rtol=0, atol=1e-9)
    assert np.all(inside | np.isclose(vt, vb, rtol=0, atol=1e-9))
    c = (np.array(si) - 1) / 2.0
    idx = np.argwhere(inside)
    r = 30.0 * np.sqrt(((idx - c) ** 2).sum(axis=1))
    assert r.max() <= 1000.0
    # every node within 1 km is inside: the sphere's node count
    I, J, K = np.meshgrid(*[np.arange(a) for a in si], indexing="ij")
    assert inside.sum() == int((30.0 * np.sqrt((I - c[0]) ** 2 + (J - c[1]) ** 2 + (K - c[2]) ** 2) <= 1000.0).sum())
    assert np.allclose(w.v[10:-10, 10:-10, 10:-10], ndimage.gaussian_filter(vb, 6.0, mode="nearest"), rtol=0,
                       atol=1e-9)
    assert len(w.src) == 64 and len(w.rec) == 48 * 48
    assert set(w.src[:, 2]) == {10} and set(w.rec[:, 2]) == {10}


def test_salt_320x320x160_recipe():
    w = W.c5_salt()
    assert w.n == (320, 320, 160) and w.h == 15.0 and w.npml == 10 and w.freq == 10.0 and w.stencil == "27pt"
    si = W.interior_shape(w.n, w.npml)
    vt = w.v_true[10:-10, 10:-10, 10:-10]
    vb = W.layered_velocity(si, 5, 1500.0, 3500.0, 2.0)
    body = vt == 4500.0
    assert np.all(body | (vt == vb))
    g = [np.arange(a) / (a - 1) for a in si]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    e = ((X - 0.5) / 0.30) ** 2 + ((Y - 0.5) / 0.25) ** 2 + ((Z - 0.55) / 0.20) ** 2
    assert np.array_equal(body, e <= 1.0)
    assert np.allclose(w.v[10:-10, 10:-10, 10:-10], ndimage.gaussian_filter(vt, 4.0, mode="nearest"), rtol=0,
                       atol=1e-9)
    assert len(w.src) == 8 and set(w.src[:, 2]) == {10}
    # receivers on every interior node of the first interior plane
    assert len(w.rec) == 300 * 300 and len({tuple(p) for p in w.rec.tolist()}) == 300 * 300
    assert w.rec[:, :2].min() == 10 and w.rec[:, :2].max() == 309 and set(w.rec[:, 2]) == {10}
