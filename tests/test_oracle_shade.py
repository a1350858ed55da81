"""Pins of the oracle's shading of splat winners (Sec. 5, Blinn-Phong from
the packed normals): closed forms for a normal facing the light, a light at
grazing angle, the two-sided flip, the specular power against fp64, and the
normal decoding against the exact direction it packs."""
from __future__ import annotations

import math

import numpy as np

from paper_2211_15460_amd import scenes as S


def _one(orc, w2, rgba, light):
    frag = np.array([[0, rgba, w2, 0]], np.uint32)
    zb = np.zeros((1, 1, 1), np.uint64)                   # fragment 0 at depth bits 0
    return orc.shade(frag, zb, np.asarray(light, np.float32).reshape(1, 13))[0, 0, 0]


def _light(L, V, H, ka, kd, ks, shine):
    return list(L) + list(V) + list(H) + [ka, kd, ks, float(shine)]


def test_facing_light_closed_form(orc):
    rgba = 0xFF336699
    c = np.array([0x99, 0x66, 0x33], np.float64) / 255
    z = (0.0, 0.0, 1.0)
    out = _one(orc, 0, rgba, _light(z, z, z, 0.25, 0.5, 0.125, 5))
    assert np.allclose(out[:3], c * 0.75 + 0.125, atol=1e-6) and out[3] == 1.0


def test_grazing_light_keeps_ambient(orc):
    rgba = 0xFF336699
    c = np.array([0x99, 0x66, 0x33], np.float64) / 255
    out = _one(orc, 0, rgba, _light((1, 0, 0), (0, 0, 1), (0.7071068, 0, 0.7071068), 0.25, 0.5, 0.125, 3))
    assert np.allclose(out[:3], c * 0.25, atol=1e-7)


def test_back_facing_normal_is_flipped(orc):
    down = orc.oct_encode(0, 0, -1)
    z = (0.0, 0.0, 1.0)
    a = _one(orc, 0, 0xFF808080, _light(z, z, z, 0.1, 0.6, 0.3, 2))
    b = _one(orc, down, 0xFF808080, _light(z, z, z, 0.1, 0.6, 0.3, 2))
    assert np.array_equal(a, b)


def test_specular_power(orc):
    th = 0.3
    H = (math.sin(th), 0.0, math.cos(th))
    for k in (0, 1, 4, 7):
        out = _one(orc, 0, 0xFF000000, _light((0, 0, 1), (0, 0, 1), H, 0.0, 0.0, 1.0, k))
        assert abs(out[0] - math.cos(th) ** (2 ** k)) < 2e-6 * 2 ** k


def test_decoded_normals_follow_the_packed_direction(orc):
    """With L = V = n the diffuse term is n_decoded . n, which the octahedral
    quantisation keeps within 1e-4 of 1; with L along an axis it is that
    component of the decoded normal."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        n = np.round(v * 2 ** 20).astype(np.int64)
        w2 = orc.oct_encode(int(n[0]), int(n[1]), int(n[2]))
        u = n / np.linalg.norm(n)
        out = _one(orc, w2, 0xFFFFFFFF, _light(u, u, u, 0.0, 1.0, 0.0, 0))
        assert abs(out[0] - 1.0) < 1e-4
        for ax in range(3):
            e = np.zeros(3)
            e[ax] = 1.0
            out = _one(orc, w2, 0xFFFFFFFF, _light(e, u, u, 0.0, 1.0, 0.0, 0))
            assert abs(out[0] - max(u[ax], 0.0)) < 2e-4


def test_empty_pixels_stay_zero(orc):
    zb = np.full((2, 3, 4), np.uint64(2 ** 64 - 1), np.uint64)
    out = orc.shade(np.zeros((1, 4), np.uint32), zb, np.zeros((2, 13), np.float32))
    assert not out.any()
