"""CPU tests of libpm.so: every symbol of include/pm.h is exported, argument
validation, and the host FP64 tables (growth, BullFrog, spectrum amplitude)
against the oracle.  No device work is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth
from oracle import cosmo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2510_05206_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    hdr = open(os.path.join(ROOT, "include", "pm.h")).read()
    names = set(re.findall(r"\b(pm_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 18
    for n in sorted(names):
        assert hasattr(lib, n), n


def _create(lib, **kw):
    from paper_2510_05206_amd import Config
    cfg = Config(**kw).to_c()
    ctx = C.c_void_p()
    st = lib.pm_create(C.byref(cfg), C.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("bad", [dict(n_p=24), dict(n_g=16, n_p=32), dict(n_g=512, n_p=32),
                                 dict(n_steps=0), dict(batch=0), dict(batch=65), dict(mak=5),
                                 dict(mak=4, grad_order=6), dict(lpt_order=3), dict(lpt_order=2, n_p=32, n_g=32),
                                 dict(stepper="fastpm", time_var="a", n_steps=0),
                                 dict(grad_order=3), dict(a_end=0.01), dict(box=-1.0)])
def test_invalid_configs_are_rejected(lib, bad):
    st, ctx = _create(lib, **bad)
    assert st == -1 and not ctx.value


def test_unbound_context_reports_state_error(lib):
    st, ctx = _create(lib, **synth.C1)
    assert st == 0
    assert lib.pm_run(ctx) == -4
    assert b"not bound" in lib.pm_last_error(ctx)
    assert lib.pm_workspace_bytes(ctx, 1) > lib.pm_workspace_bytes(ctx, 0) > 0
    lib.pm_destroy(ctx)


@pytest.mark.parametrize("wl", ["C1", "C2", "C4"])
def test_host_schedule_matches_oracle(lib, wl):
    d = getattr(synth, wl)
    st, ctx = _create(lib, **d)
    assert st == 0
    n = d["n_steps"]
    out = np.zeros((n, 8))
    assert lib.pm_schedule(ctx, 0, out.ctypes.data_as(C.c_void_p)) == 0
    ref = cosmo.bullfrog_steps(d["omega_m"], d["a_start"], d["a_end"], n)
    for row, s in zip(out, ref):
        exp = [s.D_n, s.D_half, s.D_np1, s.alpha, s.beta, s.tau1, s.tau2, s.s]
        assert np.allclose(row, exp, rtol=1e-9, atol=1e-13), (row, exp)
    desc = np.zeros(3)
    lib.pm_describe(ctx, desc.ctypes.data_as(C.c_void_p))
    assert abs(desc[0] / cosmo.D_of_a(d["omega_m"], d["a_start"]) - 1) < 1e-10
    assert abs(desc[1] / cosmo.D_of_a(d["omega_m"], 1.0) - 1) < 1e-10
    prob = synth.oracle_problem(d)
    assert abs(desc[2] / prob.spectrum_fn().amp - 1) < 1e-8
    lib.pm_destroy(ctx)


@pytest.mark.parametrize("stepper,tv,om", [("fastpm", "D", 0.31), ("bullfrog", "a", 0.31), ("fastpm", "lna", 0.31),
                                           ("bullfrog", "lna", 0.31), ("bullfrog", "superconft", 0.31),
                                           ("leapfrog", "a", 0.31), ("leapfrog", "superconft", 0.31),
                                           ("leapfrog", "lna", 1.0), ("fastpm", "superconft", 1.0)])
def test_host_schedule_variants_match_oracle(lib, stepper, tv, om):
    d = dict(synth.C2, stepper=stepper, time_var=tv, omega_m=om)
    st, ctx = _create(lib, **d)
    assert st == 0
    n = d["n_steps"]
    out = np.zeros((n, 8))
    assert lib.pm_schedule(ctx, 0, out.ctypes.data_as(C.c_void_p)) == 0
    ref = cosmo.step_table(d["omega_m"], d["a_start"], d["a_end"], n, stepper, tv)
    for row, s in zip(out, ref):
        exp = [s.D_n, s.D_half, s.D_np1, s.alpha, s.beta, s.tau1, s.tau2, s.s]
        assert np.allclose(row, exp, rtol=1e-9, atol=1e-13), (row, exp)
    lib.pm_destroy(ctx)


def test_serving_admission_respects_the_hbm_budget():
    from paper_2510_05206_amd import serve
    plan = serve.plan_batches(20e9, 16)
    per = {(k, n): serve.workspace_bytes(serve.shape_config(n, 1), k == "grad") for (k, n) in plan}
    used = sum(B * per[key] for key, B in plan.items())
    # each bucket keeps at least one slot; beyond that the plan fits the budget
    assert used <= max(20e9, sum(per.values())) * 1.0001
    assert all(B >= 1 for B in plan.values())
    # memory of the adjoint does not grow with the number of steps
    a = serve.workspace_bytes(serve.shape_config(64, 1, max_steps=5), True)
    b = serve.workspace_bytes(serve.shape_config(64, 1, max_steps=20), True)
    assert a == b
