"""The C-ABI library loads and exports every declared entry point; host-only
entry points and argument validation work without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2608_07580_amd as ff
import scenegen

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "firefit.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ff_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ff.LIB_PATH):
        from paper_2608_07580_amd import build
        build.build()
    return ff.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 14
    assert set(names) == set(ff.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_version_and_status_strings(L):
    assert "firefit" in ff.version()
    assert L.ff_status_string(ff.FF_EINVAL).decode() == "invalid argument"


def test_gauss_hermite_library_matches_oracle(L, oracle_mod):
    """The library's rule (sign-change bracketing + Newton, weights from
    p_{q-1}) against the oracle's (Golub-Welsch + Christoffel): two
    independent algorithms for the same nodes and weights."""
    for q in (8, 16, 24, 32, 48, 64):
        x, w = ff.gauss_hermite(q)
        xo, wo = oracle_mod.gauss_hermite(q)
        np.testing.assert_allclose(x, xo, atol=2e-14)
        np.testing.assert_allclose(w, wo, rtol=1e-12)


def oracle_options():
    import oracle
    return oracle.LMOptions()


def test_default_prior_and_options(L):
    for model in (1, 2):
        p = ff.default_prior(model)
        lo, hi, x0 = scenegen.default_prior(model)
        np.testing.assert_array_equal(p.lo, lo)
        np.testing.assert_array_equal(p.hi, hi)
        np.testing.assert_array_equal(p.x0, x0)
    o = ff.default_options()
    assert (o.max_iter, o.n_quad, o.precision) == (50, 32, ff.PRECISION_FP32)
    assert (o.lanes_per_pixel, o.fallback, o.ftol) == (1, 1, 1e-8)
    ora = oracle_options()
    assert (o.ftol, o.ftol_undetected, o.f_detect, o.xtol, o.gtol, o.kappa, o.tau) == \
        (ora.ftol, ora.ftol_undetected, ora.f_detect, ora.xtol, ora.gtol, ora.kappa, ora.tau)
    with pytest.raises(ff.FirefitError):
        ff.default_prior(7)


def test_argument_errors_return_einval_before_any_launch(L):
    # NULL scene / bad sizes: validated on the host
    assert L.ff_forward(None, 1, 0, 32, None, 10, None, None, None) == ff.FF_EINVAL
    assert L.ff_forward(None, 3, 0, 32, None, 10, None, None, None) == ff.FF_EINVAL
    pr = ff.default_prior(1).to_c()
    o = ff.default_options()
    assert L.ff_retrieve_batch(None, None, None, -1, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_EINVAL
    assert L.ff_retrieve_batch(None, None, None, 0, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_OK
    assert L.ff_retrieve_scene(None, None, 0, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_EINVAL
    assert "NULL" in ff.lib().ff_last_error().decode()
    x = np.empty(4)
    assert L.ff_gauss_hermite(0, x.ctypes.data_as(C.POINTER(C.c_double)), x.ctypes.data_as(C.POINTER(C.c_double))) == ff.FF_EINVAL


def test_noalloc_retrieval_rejects_bad_arguments_on_the_host(L):
    """The allocation-free entry point validates like ff_retrieve_batch and
    refuses more scenes than its fixed array holds descriptors for."""
    pr = ff.default_prior(1).to_c()
    o = ff.default_options()
    n = ff.NOALLOC_MAX_SCENES + 1
    fake = (C.c_void_p * n)(*([1] * n))
    P = (C.c_int64 * n)(*([4] * n))
    outs = (ff.ffOutputs * n)()
    f = L.ff_retrieve_batch_noalloc
    assert f(fake, fake, P, n, C.byref(pr), None, C.byref(o), outs, None, None) == ff.FF_EINVAL
    assert "FF_NOALLOC_MAX_SCENES" in L.ff_last_error().decode()
    assert f(None, None, None, -1, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_EINVAL
    assert f(None, None, None, 0, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_OK
    assert f(None, None, None, 1, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_EINVAL
    assert "NULL" in L.ff_last_error().decode()
    ob = ff.default_options(lanes_per_pixel=3)
    assert f(fake, fake, P, 1, C.byref(pr), None, C.byref(ob), outs, None, None) == ff.FF_EINVAL


def test_tune_rejects_bad_arguments_on_the_host(L):
    pr = ff.default_prior(1).to_c()
    o = ff.default_options()
    ms = C.c_double(0)
    assert L.ff_tune(None, None, None, 0, C.byref(pr), None, C.byref(o), None, None, 0, C.byref(ms), None) == ff.FF_EINVAL
    assert L.ff_tune(None, None, None, 1, None, None, C.byref(o), None, None, 0, C.byref(ms), None) == ff.FF_EINVAL


def test_adam_defaults_are_the_oracles_paper_schedule(L, oracle_mod):
    """ff_adam_options_default and the oracle's paper_stages are written
    separately from the same reading of Sec. 2.5."""
    for model in (1, 2):
        p = ff.default_prior(model)
        o = ff.adam_options(p)
        assert (o.beta1, o.beta2, o.eps) == (oracle_mod.ADAM_BETA1, oracle_mod.ADAM_BETA2, oracle_mod.ADAM_EPS)
        want = oracle_mod.paper_stages(model, p.lo, p.hi, p.x0)
        assert o.n_stages == len(want)
        n = ff.N_STATE[model]
        for k, w in enumerate(want):
            s = o.stage[k]
            assert (s.steps, s.lr, s.clip_norm) == (w.steps, w.lr, w.clip)
            assert s.free_mask == sum(1 << j for j in w.free)
            for j in w.free:
                assert (s.window_lo_nm[j], s.window_hi_nm[j]) == w.window[j]
            zs = w.zset or {}
            for j in range(n):
                if j in zs:
                    assert s.z_start[j] == pytest.approx(zs[j], abs=1e-15)
                else:
                    assert np.isnan(s.z_start[j])


def test_adam_rejects_bad_options_on_the_host(L):
    pr = ff.default_prior(1).to_c()
    fake = (C.c_void_p * 1)(1)
    rad = (C.c_void_p * 1)(1)
    P = (C.c_int64 * 1)(4)
    outs = (ff.ffOutputs * 1)()

    def call(o):
        return L.ff_adam_retrieve_batch(fake, rad, P, 1, C.byref(pr), None, C.byref(o), outs, None, None)

    bad = []
    o = ff.adam_options(); o.stage[0].lr = 0.0; bad.append(o)
    o = ff.adam_options(); o.eps = 0.0; bad.append(o)
    o = ff.adam_options(); o.beta2 = 1.0; bad.append(o)
    o = ff.adam_options(); o.n_stages = 5; bad.append(o)
    o = ff.adam_options(); o.stage[1].free_mask = 1 << 6; bad.append(o)     # model 1 has 5 variables
    o = ff.adam_options(); o.stage[0].window_lo_nm[0] = 3000.0; bad.append(o)
    o = ff.adam_options(); o.stage[0].steps = -1; bad.append(o)
    o = ff.adam_options(); o.lanes_per_pixel = 3; bad.append(o)
    o = ff.adam_options(); o.stage[0].z_start[1] = float("inf"); bad.append(o)
    for o in bad:
        assert call(o) == ff.FF_EINVAL, ff.lib().ff_last_error()
    o = ff.adam_options()
    assert L.ff_adam_retrieve_batch(None, None, None, 0, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_OK
    assert L.ff_adam_retrieve_batch(None, None, None, -1, C.byref(pr), None, C.byref(o), None, None, None) == ff.FF_EINVAL


def test_front_end_rejects_bad_arguments_on_the_host(L):
    pr = ff.default_prior(1).to_c()
    o = ff.default_options()
    outs = ff.ffOutputs()
    one = C.c_void_p(8)
    assert L.ff_hfdi_candidates(None, one, 4, -0.1, None, one, one, None) == ff.FF_EINVAL
    assert L.ff_retrieve_listed(None, one, 4, one, one, C.byref(pr), None, C.byref(o), C.byref(outs), None,
                                None) == ff.FF_EINVAL
    # the network on listed rows: a NULL network is refused before any launch
    assert L.ff_mlp_infer_listed(None, one, 4, one, 2, one, None) == ff.FF_EINVAL
    assert "NULL network" in L.ff_last_error().decode()


def test_checkpoint_errors_on_the_host(L, tmp_path):
    """ff_warmstart_load refuses a missing or foreign file before touching a
    device; NULL arguments are refused."""
    h = C.c_void_p()
    assert L.ff_warmstart_load(str(tmp_path / "none.ffws").encode(), C.byref(h)) == ff.FF_EINVAL
    bad = tmp_path / "bad.ffws"
    bad.write_bytes(b"NOPE" + bytes(64))
    assert L.ff_warmstart_load(str(bad).encode(), C.byref(h)) == ff.FF_EINVAL
    assert "not a warm-start checkpoint" in L.ff_last_error().decode()
    trunc = tmp_path / "trunc.ffws"
    trunc.write_bytes(b"FFWS" + (1).to_bytes(4, "little"))
    assert L.ff_warmstart_load(str(trunc).encode(), C.byref(h)) == ff.FF_EINVAL
    assert L.ff_warmstart_load(None, C.byref(h)) == ff.FF_EINVAL
    assert L.ff_warmstart_save(None, str(bad).encode()) == ff.FF_EINVAL
    assert L.ff_mlp_steps_done(None) == -1
    pr = ff.default_prior(1).to_c()
    assert L.ff_mlp_train_span(None, None, C.byref(pr), 10, 0, 10, 64, 1, 300.0, 0.0, 1e-3, 1e-5, None,
                               None) == ff.FF_EINVAL
