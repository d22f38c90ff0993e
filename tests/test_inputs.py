"""The seeded workload generators: determinism, shapes and the properties of the recipes."""
import numpy as np

from oracle import ism_oracle as O
from paper_1309_7128_amd import inputs


def test_uniform_faces_deterministic_and_shaped():
    u1, v1 = inputs.uniform_faces(1, 16, 8)
    u2, v2 = inputs.uniform_faces(1, 16, 8)
    assert u1.shape == (8, 17) and v1.shape == (9, 16)
    np.testing.assert_array_equal(u1, u2)
    np.testing.assert_array_equal(v1, v2)
    assert u1.min() >= -1 and u1.max() <= 1


def test_smooth64_noise_and_smoothness():
    u, v = inputs.smooth64(2, 64, 64, noise_sigma=0.0)
    un, vn = inputs.smooth64(2, 64, 64)
    assert u.shape == (64, 65) and v.shape == (65, 64)
    d = np.concatenate([(un - u).ravel(), (vn - v).ravel()])
    assert 0.8e-3 < d.std() < 1.2e-3
    # the noise-free field is band-limited to |k| <= 32: its 2D spectrum on a 64-point
    # periodic sampling has no energy above that radius
    f = np.abs(np.fft.fft2(u[:, :64]))
    k = np.fft.fftfreq(64, 1 / 64)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    assert f[kk > 32.5].max() < 1e-9 * f.max()


def test_jet_base_flow_is_divergence_free_and_perturbation_rms():
    nx, ny, lx, ly = 64, 128, 0.5, 1.0
    u, v = inputs.jet(4, nx, ny, lx, ly, rms=0.0 + 1e-300)
    b = O.div(u, v, lx / nx, O.PERIODIC)
    assert np.abs(b).max() < 1e-12
    assert abs(u.max() - 1.0) < 0.02  # peak speed 1
    u1, v1 = inputs.jet(4, nx, ny, lx, ly)
    pert = np.concatenate([(u1 - u).ravel(), v1.ravel()])
    assert abs(np.sqrt(np.mean(pert**2)) - 0.05) < 1e-12
    assert np.all(v1[0] == 0) and np.all(v1[-1] == 0)
    # step t shifts the perturbation by t cells in +x
    u2, v2 = inputs.jet(4, nx, ny, lx, ly, step=3)
    np.testing.assert_allclose((u2 - u)[:, 3:], (u1 - u)[:, :-3], atol=1e-12)


def test_workload_table():
    w = inputs.WORKLOADS["jet4096x8192_mixed"]
    assert w.u_shape == (8192, 4096) and abs(w.h - 1 / 8192) < 1e-18
    assert inputs.WORKLOADS["cavity8192_mixed"].coarsen == 32
