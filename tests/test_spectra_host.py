"""Host logic of the excitation and spectrum entry points (no GPU needed):
the field shapes against the oracle's, and argument checks that must fail
before any device work."""
import ctypes
import os

import numpy as np
import pytest

from oracle import spectra as sp


@pytest.fixture(scope="module")
def tdfe():
    from paper_1810_13130_amd import tdfe as T
    if not os.path.exists(T.LIB_PATH):
        pytest.skip("libtdfe.so not built")
    T.load()
    return T


def test_field_shapes_match_oracle(tdfe):
    t = np.linspace(-2.0, 1100.0, 20001)
    g = tdfe.field_samples(tdfe.FIELD_GAUSSIAN, (2e-5, 3.0, 0.2), t)
    assert np.abs(g - sp.field_gaussian(t, 2e-5, 3.0, 0.2)).max() <= 1e-15 * 2e-5
    om = 0.03
    T = 5 * 2 * np.pi / om
    l = tdfe.field_samples(tdfe.FIELD_SIN2, (0.01, om, T), t)
    assert np.abs(l - sp.field_sin2(t, 0.01, om, T)).max() <= 1e-15 * 0.01
    assert l[t > T].tolist() == [0.0] * int(np.sum(t > T)) and l[t < 0].tolist() == [0.0] * int(np.sum(t < 0))


def test_field_shape_errors(tdfe):
    with pytest.raises(tdfe.TdfeError):
        tdfe.field_samples(7, (1.0, 0.0, 1.0), [0.0])
    with pytest.raises(tdfe.TdfeError):
        tdfe.field_samples(tdfe.FIELD_GAUSSIAN, (1.0, 0.0, 0.0), [0.0])
    with pytest.raises(tdfe.TdfeError):
        tdfe.field_samples(tdfe.FIELD_SIN2, (1.0, np.nan, 1.0), [0.0])


def test_spectrum_argument_checks(tdfe):
    lib = tdfe.load()
    p = ctypes.c_void_p(4096)  # never dereferenced: the calls must fail on the host
    E = tdfe.EINVAL
    assert lib.tdfe_absorption_spectrum(p, None, 1, 0.1, 1e-3, 0.0, p, 4, p, None) == E  # n_t < 2
    assert lib.tdfe_absorption_spectrum(p, None, 10, 0.0, 1e-3, 0.0, p, 4, p, None) == E  # dt
    assert lib.tdfe_absorption_spectrum(p, None, 10, 0.1, 1e-3, -1.0, p, 4, p, None) == E  # alpha
    assert lib.tdfe_absorption_spectrum(p, None, 10, 0.1, 0.0, 0.0, p, 4, p, None) == E  # zero kick
    assert lib.tdfe_absorption_spectrum(None, None, 10, 0.1, 1e-3, 0.0, p, 4, p, None) == E
    assert lib.tdfe_absorption_spectrum(p, None, 10, 0.1, 1e-3, 0.0, p, 0, p, None) == tdfe.OK  # nothing to do
    assert lib.tdfe_power_spectrum(p, 2, 0.1, p, 4, p, None) == E
    assert lib.tdfe_power_spectrum(p, 10, -0.1, p, 4, p, None) == E
    assert lib.tdfe_power_spectrum(p, 10, 0.1, None, 4, p, None) == E


def test_field_direction_and_kick_checks(tdfe):
    import workloads as W
    lib = tdfe.load()
    d = tdfe.MeshDesc()
    d.p, d.nq = 2, 3
    d.ncell[0], d.ncell[1], d.ncell[2] = 2, 2, 2
    v = np.ascontiguousarray(W.box_vertices(-1.0, 1.0, (2, 2, 2)).reshape(-1))
    d.vertices = v.ctypes.data_as(tdfe._DP)
    d.n_orb_max, d.k_max, d.precision = 1, 8, 0
    h = ctypes.c_void_p()
    assert lib.tdfe_fe_mesh_setup(ctypes.byref(d), None, ctypes.byref(h)) == 0
    zero = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    bad = (ctypes.c_double * 3)(1.0, float("inf"), 0.0)
    ok = (ctypes.c_double * 3)(1.0, 0.0, 0.0)
    assert lib.tdfe_set_field_direction(h, zero) == tdfe.EINVAL
    assert lib.tdfe_set_field_direction(h, bad) == tdfe.EINVAL
    assert lib.tdfe_set_field_direction(h, ok) == tdfe.OK
    assert lib.tdfe_kick(h, ctypes.c_void_p(4096), 1, 1e-3) == tdfe.ESTATE
    assert lib.tdfe_kick(h, ctypes.c_void_p(4096), 2, 1e-3) == tdfe.EINVAL
    assert lib.tdfe_kick(h, ctypes.c_void_p(4096), 1, float("nan")) == tdfe.EINVAL
    lib.tdfe_destroy(h)


def test_adaptive_axes_description_checks(tdfe):
    lib = tdfe.load()
    R = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    one = (ctypes.c_double * 1)(1.0)
    d = tdfe.AdaptDesc()
    d.p, d.lo, d.hi, d.n_atoms, d.R, d.Z, d.s_orb, d.a_pot, d.n_elem, d.samples = 4, -1.0, 1.0, 1, R, one, one, one, 100.0, 17
    nb = ctypes.c_size_t()
    assert lib.tdfe_adaptive_axes_query(ctypes.byref(d), ctypes.byref(nb)) == 0 and nb.value >= 8 * 17 ** 3
    for field, bad in (("p", 9), ("hi", -1.0), ("n_atoms", 0), ("n_elem", 0.5), ("samples", 2)):
        old = getattr(d, field)
        setattr(d, field, bad)
        assert lib.tdfe_adaptive_axes_query(ctypes.byref(d), ctypes.byref(nb)) == tdfe.EINVAL, field
        setattr(d, field, old)
    zero = (ctypes.c_double * 1)(0.0)
    d.s_orb = zero
    assert lib.tdfe_adaptive_axes_query(ctypes.byref(d), ctypes.byref(nb)) == tdfe.EINVAL


def test_adaptive_axes_static_checks_before_device_work(tdfe):
    # the allocation-free variant refuses a bad description or a sample grid
    # whose scratch exceeds its static array before any device call
    lib = tdfe.load()
    R = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    one = (ctypes.c_double * 1)(1.0)
    d = tdfe.AdaptDesc()
    d.p, d.lo, d.hi, d.n_atoms, d.R, d.Z, d.s_orb, d.a_pot, d.n_elem, d.samples = 4, -1.0, 1.0, 1, R, one, one, one, 100.0, 161
    axes = (ctypes.c_double * 30)()
    nc = (ctypes.c_int * 3)()
    E = ctypes.c_double()
    assert lib.tdfe_adaptive_axes_static(ctypes.byref(d), None, 9, axes, nc, ctypes.byref(E)) == tdfe.ENOMEM
    nb = ctypes.c_size_t()
    assert lib.tdfe_adaptive_axes_query(ctypes.byref(d), ctypes.byref(nb)) == 0 and nb.value > 32 * 1024 * 1024
    d.samples = 160
    assert lib.tdfe_adaptive_axes_query(ctypes.byref(d), ctypes.byref(nb)) == 0 and nb.value <= 32 * 1024 * 1024
    d.p = 9
    assert lib.tdfe_adaptive_axes_static(ctypes.byref(d), None, 9, axes, nc, ctypes.byref(E)) == tdfe.EINVAL
    d.p = 4
    assert lib.tdfe_adaptive_axes_static(ctypes.byref(d), None, 0, axes, nc, ctypes.byref(E)) == tdfe.EINVAL


def test_tridiag_expm_checks_before_device_work(tdfe):
    lib = tdfe.load()
    nb = ctypes.c_size_t()
    assert lib.tdfe_tridiag_expm_query(0, ctypes.byref(nb)) == tdfe.EINVAL
    assert lib.tdfe_tridiag_expm_query(1025, ctypes.byref(nb)) == tdfe.EINVAL
    assert lib.tdfe_tridiag_expm_query(1024, ctypes.byref(nb)) == 0 and nb.value > 8 * 65536
    fake = ctypes.c_void_p(4096)
    m = ctypes.c_int()
    # a scratch below the queried size is refused before any launch
    assert lib.tdfe_tridiag_expm(fake, fake, 10, 0.1, fake, fake, 16, None, ctypes.byref(m)) == tdfe.ENOMEM
    assert lib.tdfe_tridiag_expm(fake, None, 10, 0.1, fake, fake, nb.value, None, ctypes.byref(m)) == tdfe.EINVAL
    assert lib.tdfe_tridiag_expm(fake, fake, 10, float("inf"), fake, fake, nb.value, None, None) == tdfe.EINVAL
