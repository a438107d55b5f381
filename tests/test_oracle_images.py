"""Pins of the oracle's method of images for a traction-free surface (CPU).

In anti-plane deformation a traction-free line y = y0 is the even continuation of
the displacement across it (the construction of the paper's BP1-FD check,
Appendix A): every source fault acts also through its mirror image.

* the traction on a receiver lying on the surface line vanishes, lag by lag and in
  the static limit, for a source and its image together (and not for the source
  alone);
* a fault that reaches the surface and its image are one fault of twice the
  length whose slip is continued symmetrically across the surface, the
  paper's construction, element by element at every lag;
* the dense operator with images sums the image pairs on the original faults'
  rates (a prescribed rate history equals the doubled-fault stress).
"""
import math

import numpy as np

import seas_inputs as SI
from oracle import geometry, interaction as I, seas

DT, CS, MU = 0.007, SI.CS, SI.MU


def test_traction_vanishes_on_the_surface():
    y0 = 0.0
    src = SI.free_surface_network(n_elem=12)[1]          # buried, dipping
    img = geometry.mirror_images([src], y0)[0]
    recv = SI.fault(0.0, y0, 0.0, 3000.0, 30)            # lies on the surface line, normal (0, -1)
    geo = geometry.discretize([recv, src, img])
    for T in (0, 3, 10, 40, 120, 400):
        Ks = I.pair_kernel(geo, 0, 1, T, DT, CS)
        Ki = I.pair_kernel(geo, 0, 2, T, DT, CS)
        scale = max(np.abs(Ks).max(), 1e-300)
        if np.abs(Ks).max() > 0:
            assert np.abs(Ks - Ki).max() <= 1e-12 * scale, T       # source plus image (sign -1): zero
    Gs = I.static_dipole(geo, 0, 1, MU)
    Gi = I.static_dipole(geo, 0, 2, MU)
    assert np.abs(Gs).max() > 1e3
    assert np.abs(Gs - Gi).max() <= 1e-12 * np.abs(Gs).max()


def test_surface_fault_and_image_are_the_doubled_fault():
    y0, n, dx = 0.0, 16, 50.0
    f1, f2 = SI.free_surface_network(n_elem=n, dx=dx, y0=y0)
    img = geometry.mirror_images([f1], y0)[0]
    L = n * dx
    doubled = SI.fault(0.0, y0, 90.0, 2 * L, 2 * n)    # from y0 - L to y0 + L, same normal as f1
    geo = geometry.discretize([f2, f1, img, doubled])
    rng = np.random.default_rng(0)
    slip = rng.standard_normal(n)
    cont = np.concatenate([slip, slip[::-1]])           # continued symmetrically across the surface
    for T in (0, 5, 20, 60, 200):
        with_img = I.pair_kernel(geo, 0, 1, T, DT, CS) @ slip - I.pair_kernel(geo, 0, 2, T, DT, CS) @ slip
        dbl = I.pair_kernel(geo, 0, 3, T, DT, CS) @ cont
        assert np.abs(with_img - dbl).max() <= 1e-11 * max(np.abs(dbl).max(), 1e-300), T
    sta = I.static_dipole(geo, 0, 1, MU) @ slip - I.static_dipole(geo, 0, 2, MU) @ slip
    assert np.allclose(sta, I.static_dipole(geo, 0, 3, MU) @ cont, rtol=1e-11, atol=0)


def test_dense_operator_with_images():
    y0, n = 0.0, 16
    faults = SI.free_surface_network(n_elem=n, y0=y0)
    p = SI.default_params(compress=0, free_surface=1, surface_y=y0)
    prob = seas.Problem(faults, p)
    assert prob.images is not None and set(prob.inter.pairs) == {(0, 1), (1, 0), (0, 2), (0, 3), (1, 2), (1, 3)}
    V = SI.prescribed_slip_rate(faults, 30, 3)
    f_img = seas.prescribed(prob, V)
    # the same sums with every image written out as its own source fault, taking the
    # negated rates of its original (slip minus the original's across the image normal)
    imgs = geometry.mirror_images(faults, y0)
    prob4 = seas.Problem(faults + imgs, SI.default_params(compress=0))
    V4 = np.concatenate([V, -V], axis=1)
    f4 = seas.prescribed(prob4, V4)
    # receivers of the real faults; their self terms agree (same faults, same slip), the
    # interaction sums gain the image pairs; the image faults' own rows are discarded
    assert np.abs(f_img - f4[:, :2 * n]).max() <= 1e-11 * np.abs(f4[:, :2 * n]).max()
