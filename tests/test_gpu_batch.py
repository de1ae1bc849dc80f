"""Uneven batches: persistent (work-queue) launches, graph replay and the
launch-sequence tuner, against the oracle.

The last test runs the full 512-orbital uneven batch (coarse dims uniform in
16..64 per axis, one Gaussian potential per orbital) in compensated float32,
persistent and graph-replayed, and checks sampled orbitals one by one
against the oracle (largest, smallest and a few others), plus the energies
of every orbital against their plain-float64 values on the GPU.
"""

import ctypes

import numpy as np
import pytest
import torch

from oracle import wavelet as W
from parity_helpers import assert_close, assert_scalar
from paper_0904_1543_amd import inputs, lib, ops

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 2e-6, "f32c": 1e-10}


NCAND = 15   # tuner candidates: 5 launch sequences x 3 tile shapes


def _tuning(plan):
    v = ctypes.c_int32()
    t = (ctypes.c_double * NCAND)()
    lib.wvl_plan_tuning(plan.h, ctypes.byref(v), t, NCAND)
    return v.value, list(t)


def _hpsi(plan, c, V):
    return plan.local_hpsi(c, V, rho=False, per_orbital=True)


@pytest.mark.parametrize("prec", ["f64", "f32", "f32c"])
def test_persistent_uneven_matches_oracle(prec):
    cs = inputs.random_uneven_case(51, 9, lo=2, hi=20)
    plan = ops.Plan(cs["dims"], prec=prec, shared_v=False, persistent=True)
    c, Vt = plan.pack(cs["C"]), plan.pack_potential(cs["V"])
    r = _hpsi(plan, c, Vt)
    ref = [W.local_hpsi_orbital(x, v)[0] for x, v in zip(cs["C"], cs["V"])]
    assert_close(plan.unpack(r["hpsi"]), ref, TOL[prec])
    ref_e = W.local_hpsi(cs["C"], cs["V"], cs["occ"], shared_v=False)
    eo = r["e_orb"].cpu().numpy()
    assert_close(eo[: plan.norb], ref_e["e_loc_orb"], TOL[prec])
    assert_close(eo[plan.norb:], ref_e["e_kin_orb"], TOL[prec])


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_persistent_equals_ordinary_launches(prec):
    """Same kernels, same arithmetic: the work order does not change any bit."""
    cs = inputs.random_uneven_case(52, 12, lo=3, hi=24)
    a = ops.Plan(cs["dims"], prec=prec, shared_v=False)
    b = ops.Plan(cs["dims"], prec=prec, shared_v=False, persistent=True)
    c, Vt = a.pack(cs["C"]), a.pack_potential(cs["V"])
    ra, rb = _hpsi(a, c, Vt), _hpsi(b, c, Vt)
    assert torch.equal(ra["hpsi"], rb["hpsi"])
    assert torch.equal(ra["e_orb"], rb["e_orb"])
    assert torch.equal(ra["energies"], rb["energies"])


def test_persistent_graph_replay_matches_eager():
    cs = inputs.random_uneven_case(53, 10, lo=3, hi=20)
    eager = ops.Plan(cs["dims"], prec="f32c", shared_v=False, persistent=True)
    graph = ops.Plan(cs["dims"], prec="f32c", shared_v=False, persistent=True, graph=True)
    c, Vt = eager.pack(cs["C"]), eager.pack_potential(cs["V"])
    ref = _hpsi(eager, c, Vt)
    out = graph.empty()
    en = torch.empty(2, dtype=torch.float64, device="cuda:0")
    eo = torch.empty(2 * graph.norb, dtype=torch.float64, device="cuda:0")
    for rep in range(4):
        out.fill_(float("nan"))
        en.zero_()
        lib.wvl_local_hpsi(graph.h, ops.ptr(c), ops.ptr(Vt), 1.0, 1.0, ops.ptr(out), None,
                           ctypes.c_void_p(en.data_ptr()), ctypes.c_void_p(en.data_ptr() + 8),
                           ops.ptr(eo), ops.ptr(graph.ws), ops.stream_handle())
        torch.cuda.synchronize()
        assert torch.equal(out, ref["hpsi"]), rep
        assert torch.equal(eo, ref["e_orb"]), rep
        assert torch.equal(en, ref["energies"]), rep
        _ = (c * 2.0).sum().item()   # unrelated eager work between replays


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_autotune_picks_a_timed_candidate(prec):
    cs = inputs.random_case(54, 4, (20, 18, 16), potential="gauss16")
    plan = ops.Plan(cs["dims"], prec=prec, autotune=True)
    variant, times = _tuning(plan)
    measured = [t for t in times if t >= 0]
    # pass-by-pass in two axis-1 tile shapes, the plane kernel at two
    # occupancies (and the float64 vector engine); no persistent shapes
    assert times[0] > 0 and times[1] > 0 and times[3] > 0 and times[6] > 0
    assert len(measured) == (5 if prec == "f64" else 4)
    assert all(times[k] < 0 for k in (2, 4, 5, 7, 8, 10, 11))
    assert variant in (0, 1, 2)
    # the kept candidate is the fastest one measured
    best = int(np.argmin([t if t >= 0 else np.inf for t in times]))
    assert plan.query(lib.WVL_Q_TUNE_BEST) == best
    seq = best // 3
    expect = {0: 0, 1: 2 if prec == "f64" else 1, 2: 2 if prec == "f64" else 1, 3: 1}[seq]
    assert variant == expect
    assert plan.query(lib.WVL_Q_XDIV) == (2 if best == 1 else 1)
    r = plan.local_hpsi(plan.pack(cs["C"]), plan.pack_potential(cs["V"]), per_orbital=True)
    ref = W.local_hpsi(cs["C"], cs["V"], cs["occ"])
    assert_close(plan.unpack(r["hpsi"]), list(ref["hpsi"]), TOL[prec])


def test_untuned_plan_reports_no_times():
    cs = inputs.random_case(55, 2, (6, 6, 6))
    plan = ops.Plan(cs["dims"], prec="f64")
    _, times = _tuning(plan)
    assert times == [-1.0] * NCAND
    assert plan.query(lib.WVL_Q_TUNE_BEST) == -1


@pytest.mark.parametrize("prec", ["f64", "f32", "f32c"])
@pytest.mark.parametrize("mode", ["plain", "persistent", "graph"])
def test_pass_by_pass_per_orbital_potential(prec, mode, monkeypatch):
    """The pass-by-pass sequence with one potential per orbital (its pointwise
    stage is the per-orbital kernel), eager, persistent and graph-replayed."""
    monkeypatch.setenv("WVL_NO_PLANE_KERNEL", "1")
    cs = inputs.random_uneven_case(56, 11, lo=2, hi=22)
    plan = ops.Plan(cs["dims"], prec=prec, shared_v=False, persistent=(mode != "plain"),
                    graph=(mode == "graph"))
    assert plan.query(lib.WVL_Q_VARIANT) == 0
    assert plan.query(lib.WVL_Q_PERSISTENT) == (mode != "plain")
    c, Vt = plan.pack(cs["C"]), plan.pack_potential(cs["V"])
    ref = W.local_hpsi(cs["C"], cs["V"], cs["occ"], shared_v=False)
    for rep in range(2 if mode == "graph" else 1):
        r = _hpsi(plan, c, Vt)
        assert_close(plan.unpack(r["hpsi"]), ref["hpsi"], TOL[prec], f"hpsi (call {rep})")
        eo = r["e_orb"].cpu().numpy()
        assert_close(eo[: plan.norb], ref["e_loc_orb"], TOL[prec], "e_pot per orbital")
        assert_close(eo[plan.norb:], ref["e_kin_orb"], TOL[prec], "e_kin per orbital")
        e = r["energies"].cpu().numpy()
        assert_scalar(e[0], float(np.sum(cs["occ"] * ref["e_loc_orb"])), TOL[prec], "E_loc")
        assert_scalar(e[1], ref["e_kin"], TOL[prec], "E_kin")


def test_uneven_512_orbital_batch_f32c_persistent_graph():
    """The 512-orbital batch through the launch sequence the tuner picks."""
    wl = inputs.workload(5)
    dims = wl["dims"]
    plan = ops.Plan(dims, prec="f32c", shared_v=False, persistent=True, graph=True,
                    autotune=True)
    print(f"tuner kept candidate {plan.query(lib.WVL_Q_TUNE_BEST)}, "
          f"variant {plan.query(lib.WVL_Q_VARIANT)}", flush=True)
    assert plan.query(lib.WVL_Q_PERSISTENT) == 1
    c = plan.pack(wl["C"])
    Vt = plan.pack_potential(wl["V"])
    out = plan.empty()
    eo = torch.empty(2 * plan.norb, dtype=torch.float64, device="cuda:0")
    for _ in range(2):
        lib.wvl_local_hpsi(plan.h, ops.ptr(c), ops.ptr(Vt), 1.0, 1.0, ops.ptr(out), None, None,
                           None, ops.ptr(eo), ops.ptr(plan.ws), ops.stream_handle())
    torch.cuda.synchronize()
    sizes = [int(np.prod(d)) for d in dims]
    sample = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 0, 137, 511})
    got = plan.to_f64(out)
    for b in sample:
        o, m = int(plan.offsets[b]), plan.M[b]
        g = got[o:o + m].cpu().numpy().reshape(inputs.fine_shape(dims[b]))
        ref = W.local_hpsi_orbital(wl["C"][b], wl["V"][b])[0]
        print(f"orbital {b} dims {dims[b]}", flush=True)
        assert_close(g, ref, TOL["f32c"], f"orbital {b}")
    # every orbital's energies against the float64 plan (itself within 1e-12 of the oracle)
    del out
    ref64 = ops.Plan(dims, prec="f64", shared_v=False)
    c64 = plan.to_f64(c)
    r64 = ref64.local_hpsi(c64, Vt, rho=False, per_orbital=True)
    assert_close(eo.cpu().numpy(), r64["e_orb"].cpu().numpy(), TOL["f32c"])
