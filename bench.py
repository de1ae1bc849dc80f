#!/usr/bin/env python3
"""Throughput of the local Hamiltonian on one MI355X, in orbital-gridpoints/s.

One step is the whole hot path over one batch: wavelet synthesis, magic
filter, density and potential product, transposed magic filter, kinetic
operator, wavelet analysis (the local H*psi of Sec. 2.4, with the density of
Sec. 2.5 and the float64 energy reductions), then the float64 overlap matrix
and the Cholesky orthonormalisation of the batch (Sec. 5 step VIII).

Workload: 256 orbitals on a periodic coarse grid of 48^3 (fine 96^3), the
precision form of the paper's method; float64 is the headline, plain float32
and compensated float32 (hi + lo planes) are reported beside it with their
measured errors against the float64 oracle.  Inputs are seeded and synthetic
and already resident in device memory when the timed region starts.

Prints one JSON line.  Options: --steps K --warmup W --gpus 1.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("orbital-gridpoints/s for local H*psi (HBM GB/s % peak), FP64 vs FP32-comp at 1e-10")
HBM_PEAK_GBS = 8000.0
ESIZE = {"f64": 8, "f32": 4, "f32c": 8}
TOL = {"f64": 1e-12, "f32": 2e-6, "f32c": 1e-10}


def algorithmic_bytes(stage, plan, variant):
    """Bytes a launch of `stage` must move for the whole batch (each value
    read or written once): a 1D pass reads its input and writes its output;
    passes that accumulate (kinetic K_{p-1}, and with the plane kernel the last
    two z passes) also read the accumulator; the plane kernel reads u and c
    and writes t and kxy; the potential stage reads psi, V and writes y and
    rho; the overlap reads the coefficients once."""
    E, es, M = plan.elems, ESIZE[plan.prec], plan.M[0]
    if stage == "xy_plane":
        return 4 * E * es
    if stage in ("ck_z", "cwt_z") and variant == 1:
        return 3 * E * es
    if stage.startswith("kin_") or stage.startswith("ck_"):
        return 3 * E * es
    if stage[:3] in ("mf_", "mft", "syn", "ana", "cw_", "cwt"):
        return 2 * E * es
    if stage == "potential":
        return 2 * E * es + 2 * M * 8
    if stage in ("overlap",):
        return E * es
    if stage == "trmm":
        return 2 * E * es
    return None


def run_precision(prec, C, V, dims, steps, warmup, sample_orbs):
    import torch
    from paper_0904_1543_amd import ops

    plan = ops.Plan(dims, prec=prec)
    c = plan.pack(C)
    Vt = plan.pack_potential(V)
    out = plan.empty()
    rho = torch.empty(plan.M[0], dtype=torch.float64, device=plan.dev)
    en = torch.empty(2, dtype=torch.float64, device=plan.dev)
    eorb = torch.empty(2 * plan.norb, dtype=torch.float64, device=plan.dev)

    import ctypes
    from paper_0904_1543_amd import lib

    def hpsi():
        lib.wvl_local_hpsi(plan.h, ops.ptr(c), ops.ptr(Vt), 1.0, 1.0, ops.ptr(out), ops.ptr(rho),
                           ctypes.c_void_p(en.data_ptr()), ctypes.c_void_p(en.data_ptr() + 8),
                           ops.ptr(eorb), ops.ptr(plan.ws), ops.stream_handle())

    def step():
        hpsi()
        plan.orthonormalize(out)

    # accuracy of this precision on sampled orbitals (untimed)
    hpsi()
    torch.cuda.synchronize()
    got = {}
    if sample_orbs:
        allo = plan.unpack(out)
        got = {b: allo[b].copy() for b in sample_orbs}
        del allo
    energies = en.cpu().numpy().copy()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(64 * (steps + 1))
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t0.record()
    for _ in range(steps):
        step()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = t0.elapsed_time(t1) / steps
    recs = plan.profile_read()
    plan.profile(0)
    plan.sync()
    # per-stage launch durations over the timed region
    stages = {}
    for name, t in recs:
        s = stages.setdefault(name, [0.0, 0])
        s[0] += t
        s[1] += 1
    table = {k: {"avg_ms": v[0] / v[1], "launches": v[1], "share": v[0] / (ms * steps)}
             for k, v in stages.items()}
    hpsi_ms = sum(v[0] for k, v in stages.items()
                  if k not in ("overlap", "cholesky", "trmm")) / steps
    v = ctypes.c_int32()
    lib.wvl_plan_tuning(plan.h, ctypes.byref(v), None, 0)
    res = dict(plan=plan, ms_per_step=ms, wall_s=wall, stages=table, hpsi_ms=hpsi_ms, got=got,
               energies=energies, variant=v.value)
    del c, Vt, out, rho
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precs", default="f64,f32c,f32")
    ap.add_argument("--cpu-orbitals", type=int, default=40,
                    help="orbitals of the batch the oracle is timed on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the orbital batch would be split across GPUs, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0904_1543_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    wl = inputs.workload(3)
    C, V, dims = wl["C"], wl["V"], wl["dims"]
    norb = len(dims)
    pts = norb * int(np.prod(inputs.fine_shape(dims[0])))
    sample = [] if args.no_cpu_baseline else [0, norb - 1]

    precs = [p for p in args.precs.split(",") if p]
    results = {}
    for prec in precs:
        print(f"[bench] {prec}: {norb} orbitals x {inputs.fine_shape(dims[0])}", file=sys.stderr,
              flush=True)
        results[prec] = run_precision(prec, C, V, dims, args.steps, args.warmup, sample)
        torch.cuda.empty_cache()

    # oracle: CPU baseline on a bounded sample, and the errors of every precision
    cpu = None
    errors = {}
    if not args.no_cpu_baseline:
        from oracle import wavelet as W
        ncpu = max(1, min(args.cpu_orbitals, norb))
        idx = sorted(set([0, norb - 1] + list(range(1, ncpu - 1))))[:ncpu]
        refs = {}
        t = time.perf_counter()
        for b in idx:
            refs[b] = W.local_hpsi_orbital(C[b], V)[0]
        tcpu = time.perf_counter() - t
        cpu = {"value": len(idx) * pts / norb / tcpu, "unit": "orbital-gridpoints/s",
               "cores": 1, "kind": "oracle",
               "sample": f"{len(idx)} of {norb} orbitals (96^3 fine grid each), plain float64 "
                         f"numpy oracle, single thread, {tcpu:.1f} s"}
        for prec, r in results.items():
            num = sum(np.sum((r["got"][b] - refs[b]) ** 2) for b in r["got"])
            den = sum(np.sum(refs[b] ** 2) for b in r["got"])
            errors[prec] = float(np.sqrt(num / den))

    head = "f64" if "f64" in results else precs[0]
    r = results[head]
    ms = r["ms_per_step"]
    # dominant kernel of the headline precision
    dom, dstat = max(r["stages"].items(), key=lambda kv: kv[1]["avg_ms"] * kv[1]["launches"])
    ab = algorithmic_bytes(dom, r["plan"], r["variant"])
    roof = None
    if ab is not None:
        gbs = ab / (dstat["avg_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_ms": round(dstat["avg_ms"], 4),
                "algorithmic_bytes": int(ab)}
    line = {
        "metric": METRIC,
        "value": pts / (ms * 1e-3),
        "unit": "orbital-gridpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": "256 orbitals, periodic coarse 48^3 (fine 96^3), local H*psi "
                               "with density and energies + float64 overlap/Cholesky "
                               "orthonormalisation", "orbitals": norb,
                   "fine_grid": list(inputs.fine_shape(dims[0])),
                   "potential": "16 periodic Gaussians", "seed": 3},
        "roofline": roof,
        "cpu_baseline": cpu,
        "precisions": {
            p: {"ms_per_step": v["ms_per_step"],
                "hpsi_variant": "plane-resident" if v["variant"] == 1 else "pass-by-pass",
                "orbital_gridpoints_per_s": pts / (v["ms_per_step"] * 1e-3),
                "hpsi_ms": v["hpsi_ms"],
                "hpsi_orbital_gridpoints_per_s": pts / (v["hpsi_ms"] * 1e-3),
                "rel_err_vs_oracle": errors.get(p),
                "tolerance": TOL[p],
                "e_loc": float(v["energies"][0]), "e_kin": float(v["energies"][1]),
                "stages": {k: {"avg_ms": round(s["avg_ms"], 4), "launches": s["launches"]}
                           for k, s in sorted(v["stages"].items(),
                                              key=lambda kv: -kv[1]["avg_ms"] * kv[1]["launches"])}}
            for p, v in results.items()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
