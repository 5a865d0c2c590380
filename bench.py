#!/usr/bin/env python3
"""Throughput benchmark of the SDF photon random walk on one MI355X.

Workload: the layered slab -- three stacked boxes 2 x 2 cm laterally,
0.01 / 0.2 / 1 cm thick (mu_a 1 / 0.2 / 0.1 /cm, mu_s 100 / 200 / 100 /cm,
g 0.8 / 0.9 / 0.9, n 1.5 / 1.4 / 1.4) in air, a normally incident pencil
beam, 1e7 packets per step, FP64 fluence on a 200^3 grid.  A step is one
smcrt_run over 1e7 packets: emission, sphere tracing, interfaces,
interactions, roulette and the fluence tally, with the scene already
resident.  Prints one JSON line.

Beside the GPU number: the fluence error against the FP64 oracle on the
first packets of the same stream, the VALU roofline of the walk kernel and
the oracle's own throughput on the host cores (a baseline, not a target).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photon packets/s at fixed fluence error vs FP64 oracle; p50/p99 request latency"
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 3.93e13 lane-ops/s

# Algorithmic VALU work per unit in lane-slots (full-rate op = 1, quarter-rate
# transcendental or 32-bit multiply-high = 4, FP64 FMA = 1):
COST = {
    "philox": 140,        # one Philox4x32-10 block
    "log": 8,             # free-path sample
    "sdf_box": 20,        # one box SDF (sphere 12, capsule 22, cylinder 25)
    "step_overhead": 12,  # min, abs, compares and the move of one sphere-tracing step
    "volume": 20,         # simulation-volume SDF per step
    "interaction": 70,    # absorption, HG, rotation, roulette (FP64 weight)
    "interface": 250,     # FP64 interface step without its SDF evaluations
    "surface_sdfs": 14,   # region SDF evaluations in one interface step (2 normals + nearest)
    "voxel": 15,          # DDA step and run merge per voxel piece
}


def slab_lane_ops(t, n_prims, coarse_interface=False):
    """lane-slots of one run from its own work counters.  An interface step
    is priced as the kernel runs it: its FP64 work, 14 SDF evaluations of
    the nearest region (two central-difference normals of 6 each, the
    distance at the snapped point and the probe), the nearest-region search
    over all primitives and the Philox block of the Fresnel draw.
    coarse_interface: the coarser price 250 + P SDF instead."""
    sdf = COST["sdf_box"]
    per_step = COST["step_overhead"] + n_prims * sdf + COST["volume"]
    emit = COST["philox"] + COST["log"] + n_prims * sdf
    inter = COST["interaction"] + COST["philox"] + COST["log"]
    surf = COST["interface"] + COST["surface_sdfs"] * sdf + n_prims * sdf + COST["philox"]
    if coarse_interface:
        surf = COST["interface"] + n_prims * sdf
    return (t["launched"] * emit + t["steps"] * per_step + t["interactions"] * inter
            + (t["interfaces"] + t["advances"]) * surf + t["voxel_pieces"] * COST["voxel"])


def measured_counters():
    """Per-launch figures of the committed rocprofv3 counter summary (HBM
    traffic, atomic requests), or {} when the kernel sources changed since
    those counters were taken."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2112_08035_amd", "csrc")
    h = hashlib.sha256()
    for f in ("walk.hip", "walk_common.h", "voxel_model.h", "layout.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    path = os.path.join(ROOT, "profiles", "walk_kernel_slab_1e7_f32_traffic.md")
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "|", "#")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != h.hexdigest()[:16]:
        return {}
    return {k: float(vals[k]) for k in ("traffic_bytes_per_launch", "atomic_requests_per_launch") if k in vals}


def measured_traffic():
    """HBM-side bytes per launch (committed counter summary), or None."""
    return measured_counters().get("traffic_bytes_per_launch")


SERVE_GRIDS = (32, 64, 128, 256)


def atomic_ceiling(key="requests_per_s"):
    """FP64 global atomic 64-byte requests per second measured on the device
    by paper_2112_08035_amd/atomic_ceiling (committed summary), or None.
    The rate is per request: the adds of one instruction that fall in one
    64-byte segment travel as one request."""
    path = os.path.join(ROOT, "profiles", "fp64_atomic_ceiling.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith(key + ":"):
            return float(line.split(":", 1)[1])
    return None


def prefix_error(smcrt, desc, seed, m, precision, geometry="sdf", engine=None, oracle_desc=None):
    """Error of the GPU path against the FP64 oracle on the same packets:
    packets [0, m) of `desc` under `seed` on both sides (the same walks, up to
    rounding; oracle_desc: the oracle's scene when it differs, e.g. the plain
    march for an over-relaxed walk), relative L2 of the fluence (and of the
    escape image when the scene has one), relative difference of the
    absorbed and escaped totals."""
    import numpy as np

    from oracle import oracle as orc
    d = dict(desc, geometry=geometry)
    eng = engine if engine is not None else smcrt.Engine(0, precision=precision)
    g = smcrt.run(d, seed, m, engine=eng, precision=precision)
    o = orc.run(dict(oracle_desc if oracle_desc is not None else desc, geometry=geometry), seed, m,
                voxel=(geometry == "voxel"))
    if engine is None:
        eng.close()

    def rel(a, b):
        nb = float(np.linalg.norm(b))
        return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))

    res = {"packets": m,
           "absorbed_relative": rel(g["absorbed"].sum(), o["absorbed"].sum()),
           "escaped_relative": rel(g["escaped_face"].sum(), o["escaped_face"].sum())}
    if g.get("fluence_raw") is not None and o.get("fluence_raw") is not None:
        res["fluence_relative_l2"] = rel(g["fluence_raw"], o["fluence_raw"])
    if "image" in g and "image" in o:
        res["image_relative_l2"] = rel(g["image"], o["image"])
    return res


def trace_parity(smcrt, workloads, precision, n=4096, cap=50):
    """Event-by-event agreement of the GPU walk with the oracle's on the
    first n packets of the layered slab (first cap events): the fraction of
    packets whose records all agree to 1e-5 (positions relative to the
    scene's extent, directions, weights, remaining path) and the diverged
    fraction (a record whose type, region or index differs)."""
    import numpy as np

    from oracle import oracle as orc
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_helpers import compare_traces, diverged_fraction, extent_of
    desc = workloads.slab_scene(n_grid=16)
    eng = smcrt.Engine(0, precision=precision)
    g = smcrt.trace(desc, 31, list(range(n)), cap, engine=eng, precision=precision)
    eng.close()
    o = [orc.trace(desc, 31, pid, cap) for pid in range(n)]
    mut = [rg["mua"] + rg["mus"] for rg in desc["regions"]]
    frac, worst, _ = compare_traces(o, g, extent_of(smcrt, desc), 1e-5, cap=cap, mut=mut)
    return {"workload": "layered slab", "packets": n, "events": cap, "agree_1e-5": frac,
            "diverged_fraction": diverged_fraction(o, g, cap),
            "worst": {k: float(v) for k, v in worst.items()}}


SERVE_BUDGET = 8 << 30  # device bytes the served requests may hold at once (outputs, tables, grids)


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fluence_z_scores(smcrt, sc, eng, precision, desc, n, Fo):
    """Per-voxel z-scores of the GPU fluence against the oracle's Fo (packets
    [0, n), seed 0), with Monte Carlo standard errors from GPU batches.
    Same packets: the GPU sum of 10 batches of [0, n) against Fo, the SE of
    that sum from the batches (floored at one packet's largest deposit, the
    voxel diagonal); the same walks put the chi-square per degree of freedom
    near 0 (at most 1.1 passes).  Independent packets: 20 batches of
    [n, 2n) against Fo, the SE of the difference from those batches (both
    sums have the batch variance times 20); the same distribution puts it
    near 1.  Both scale the mean squared z by (nu - 2)/nu, nu the batch
    degrees of freedom, so that a Student-t z averages 1."""
    import numpy as np
    lo, hi, dims = desc["grid"]["lo"], desc["grid"]["hi"], desc["grid"]["dims"]
    diag = float(np.sqrt(sum(((hi[i] - lo[i]) / dims[i]) ** 2 for i in range(3))))

    def batches(first, B):
        m = n // B
        s1 = s2 = mn = None
        for b in range(B):
            F = smcrt.run(sc, 0, m, first=first + b * m, engine=eng, precision=precision)["fluence_raw"]
            s1 = F.copy() if s1 is None else s1 + F
            s2 = F * F if s2 is None else s2 + F * F
            mn = F.copy() if mn is None else np.minimum(mn, F)
        var = np.maximum(s2 - s1 * s1 / B, 0.0) / (B - 1)
        return s1, var, mn

    B = 10
    Fg, var, _ = batches(0, B)
    se = np.sqrt(B * var)
    sel = (se > 0) | (Fg != Fo)
    z = np.abs(Fg[sel] - Fo[sel]) / np.maximum(se[sel], diag)
    same = {"batches": B, "voxels": int(sel.sum()), "within_3se": float(np.mean(z <= 3.0)),
            "max_z": float(z.max()), "chi2_per_dof": float(np.mean(z ** 2)) * (B - 3) / (B - 1)}
    B2 = 20
    Gs, var2, mn = batches(n, B2)
    keep = (mn > 0) & (Fo > 0) & (var2 > 0)  # voxels every batch reaches (elsewhere a few visits are not Gaussian)
    z2 = (Gs[keep] - Fo[keep]) ** 2 / (2.0 * B2 * var2[keep])
    nu = B2 - 1
    indep = {"batches": B2, "packets": [n, 2 * n], "voxels": int(keep.sum()),
             "within_3se": float(np.mean(np.sqrt(z2) <= 3.0)), "chi2_per_dof": float(z2.mean()) * (nu - 2) / nu}
    return {"same_packets": same, "independent_packets": indep}


def serving_capacity(smcrt, workloads, max_packets, precision, seed, n_requests=48, budget=SERVE_BUDGET):
    """Closed-loop capacity of the server on the request mix: a calibration
    stream (its own seed) submitted all at once; packets per second from
    the first submission to the last completion.  Beside it, the same
    requests run one per launch on a plain engine, one after another (the
    plain one-scene-per-launch walk the server is to beat); returns both
    rates."""
    import torch
    reqs = workloads.request_stream(seed, n_requests, 1.0, packets=(1e4, max_packets), grid_sides=SERVE_GRIDS)
    scenes = [smcrt.Scene(r["scene"]) for r in reqs]
    outs = [smcrt.Outputs(sc) for sc in scenes]
    torch.cuda.synchronize()
    sv = smcrt.Server(0, hbm_budget_bytes=budget, precision=precision)
    ids = [sv.submit(sc, r["seed"], r["n_packets"], outputs=o)[0] for r, sc, o in zip(reqs, scenes, outs)]
    for rid in ids:
        sv.wait(rid, 1200.0)
    polls = [sv.poll(rid) for rid in ids]
    sv.close()
    span = max(p[3] for p in polls) - min(p[1] for p in polls)
    total = sum(r["n_packets"] for r in reqs)
    eng = smcrt.Engine(0, precision=precision)
    smcrt.launch(eng, scenes[0], 1, 10_000, outputs=smcrt.Outputs(scenes[0]))  # warm-up
    for o in outs:
        o.zero_()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for r, sc, o in zip(reqs, scenes, outs):
        smcrt.launch(eng, sc, r["seed"], r["n_packets"], outputs=o)
    torch.cuda.synchronize()
    plain = total / (time.perf_counter() - t)
    eng.close()
    return total / span, plain


def serving(smcrt, workloads, n_requests, rate_hz, max_packets, precision, seed=2112, load=0.7, budget=SERVE_BUDGET):
    """Continuous-batching leg on the resident server: a seeded Poisson
    stream of requests drawn from the four scene families (randomised
    optical properties, grids 32^3 to 256^3, packets log-uniform from 1e4 to
    max_packets) submitted at their arrival times to one server with an
    HBM budget (8 GiB unless given; the peak bytes held are reported, so a
    run shows whether the budget bound); latency = completion - submission.
    Without a
    given rate, arrivals are set for the offered load `load` (mean packets
    per request x rate / measured closed-loop capacity).  Four check
    requests (2000 packets, one per family) ride in the stream and are
    compared with the FP64 oracle on the same packets."""
    import math

    import numpy as np
    import torch

    from oracle import oracle as orc
    mean_packets = (max_packets - 1e4) / math.log(max_packets / 1e4)  # log-uniform on [1e4, max]
    capacity, one_per_launch = serving_capacity(smcrt, workloads, max_packets, precision, seed + 1, budget=budget)
    progress(f"serving: closed-loop capacity {capacity:.3e} packets/s ({one_per_launch:.3e} one per launch)")
    if rate_hz <= 0:
        rate_hz = load * capacity / mean_packets
    reqs = workloads.request_stream(seed, n_requests, rate_hz, packets=(1e4, max_packets), grid_sides=SERVE_GRIDS)
    checks = [workloads.sphere_scene(32), workloads.slab_scene(32), workloads.cylinder_scene(32),
              workloads.vessel_scene(3, 1.0, n_caps=2000, n_grid=32)]
    for i, d in enumerate(checks):
        reqs.insert(1 + i * (len(reqs) // len(checks)),
                    {"id": -1 - i, "arrival": None, "scene": d, "seed": 77 + i, "n_packets": 2000})
    for i, r in enumerate(reqs):  # checks arrive with their neighbours
        if r["arrival"] is None:
            r["arrival"] = reqs[i - 1]["arrival"]
    scenes = [smcrt.Scene(r["scene"]) for r in reqs]
    outs = [smcrt.Outputs(sc) for sc in scenes]
    torch.cuda.synchronize()
    sv = smcrt.Server(0, hbm_budget_bytes=budget, precision=precision)
    t0 = time.perf_counter()
    ids = []
    peak_bytes, peak_queued, t_note = 0, 0, t0
    for r, sc, o in zip(reqs, scenes, outs):
        while True:
            delay = r["arrival"] - (time.perf_counter() - t0)
            if delay <= 0:
                break
            time.sleep(min(delay, 0.05))
            st = sv.stats()
            peak_bytes, peak_queued = max(peak_bytes, st["bytes_in_use"]), max(peak_queued, st["queued"])
        ids.append(sv.submit(sc, r["seed"], r["n_packets"], outputs=o)[0])
        if time.perf_counter() - t_note > 30:
            t_note = time.perf_counter()
            progress(f"serving: {len(ids)} of {len(reqs)} requests submitted")
    while True:
        st = sv.stats()
        peak_bytes, peak_queued = max(peak_bytes, st["bytes_in_use"]), max(peak_queued, st["queued"])
        if st["queued"] == 0 and st["active"] == 0:
            break
        time.sleep(0.05)
        if time.perf_counter() - t_note > 30:
            t_note = time.perf_counter()
            progress(f"serving: {st['queued']} queued, {st['active']} running")
    for rid in ids:
        sv.wait(rid, 1200.0)
    polls = [sv.poll(rid) for rid in ids]
    lat = np.array([p[3] - p[1] for p in polls])
    t_first = min(p[1] for p in polls)
    t_last = max(p[3] for p in polls)
    # time with at least one request submitted and not done: the union of
    # the requests' [submission, completion] intervals
    pending, open_end = 0.0, -math.inf
    for a, b in sorted((p[1], p[3]) for p in polls):
        if b > open_end:
            pending += b - max(a, open_end)
            open_end = b
    total = sum(r["n_packets"] for r in reqs)
    st = sv.stats()
    errs = []
    for r, o in zip(reqs, outs):
        if r["id"] >= 0:
            continue
        g = o.host()
        ro = orc.run(r["scene"], r["seed"], r["n_packets"])
        errs.append({"family": r["scene"]["name"], "packets": r["n_packets"],
                     "relative_l2": float(np.linalg.norm(g["fluence_raw"] - ro["fluence_raw"]) / np.linalg.norm(ro["fluence_raw"])),
                     "absorbed_relative": float(abs(g["absorbed"].sum() - ro["absorbed"].sum()) / ro["absorbed"].sum())})
    sv.close()
    return {
        "requests": len(reqs),
        "rate_hz": rate_hz,
        "capacity_packets_per_s": capacity,
        "one_per_launch_packets_per_s": one_per_launch,
        "capacity_over_one_per_launch": capacity / one_per_launch,
        "offered_load": rate_hz * mean_packets / capacity,
        "packets_range": [1e4, max_packets],
        "grid_sides": list(SERVE_GRIDS),
        "hbm_budget_bytes": budget,
        "peak_bytes_in_use": peak_bytes,
        "peak_queued": peak_queued,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "aggregate_packets_per_s": total / (t_last - t_first),
        "packets": total,
        "epochs": st["epochs"],
        "epoch_ms": 20.0,
        "packets_saved_and_resumed": st["saved_total"],
        "device_busy_fraction": st["busy_s"] / max(t_last - t_first, 1e-9),
        "device_busy_while_pending": st["busy_s"] / max(pending, 1e-9),
        "pending_fraction": pending / max(t_last - t_first, 1e-9),
        "check_requests_vs_oracle": errs,
    }


def comparator(smcrt, workloads, precision, n=100_000_000, seed=3):
    """Voxelised vs SDF geometry (the comparison of Sec. 3) on the curved
    vessel workload: a capped-cylinder vessel across a 1 cm tissue cube,
    top-hat beam, 256^3 FP64 grid.  Both models walk the same packets and
    seeds; reported are each one's packets/s (whole run: tables, grids,
    voxelisation, walk) and the voxel model's deviation from the SDF model's
    tallies, beside the SDF model's own seed-to-seed Monte Carlo spread."""
    import numpy as np
    import torch
    desc = workloads.cylinder_scene(256)
    res, outs = {}, {}
    for geom, sd in (("sdf", seed), ("voxel", seed), ("sdf_reseeded", seed + 1)):
        eng = smcrt.Engine(0, precision=precision)
        sc = smcrt.Scene(dict(desc, geometry="voxel" if geom == "voxel" else "sdf"))
        out = smcrt.Outputs(sc)
        smcrt.launch(eng, sc, seed + 100, 1_000_000, outputs=out)  # warm-up
        torch.cuda.synchronize()
        out.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        smcrt.launch(eng, sc, sd, n, outputs=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        outs[geom] = out.host()
        if geom != "sdf_reseeded":
            res[geom + "_packets_per_s"] = n / dt
        eng.close()

    def coarse(F):  # 32^3 blocks of 8^3 voxels
        return F.reshape(32, 8, 32, 8, 32, 8).sum(axis=(1, 3, 5))

    def rel_l2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    Fs, Fv, Fr = (outs[k]["fluence_raw"] for k in ("sdf", "voxel", "sdf_reseeded"))
    res.update({
        "workload": "capped-cylinder vessel (r 0.05 cm) in a 1 cm tissue cube, disc beam, 256^3 grid",
        "packets": n,
        "fluence_relative_l2_voxel_vs_sdf": rel_l2(Fv, Fs),
        "fluence_relative_l2_voxel_vs_sdf_32cubed": rel_l2(coarse(Fv), coarse(Fs)),
        "fluence_relative_l2_sdf_seed_to_seed": rel_l2(Fr, Fs),
        "fluence_relative_l2_sdf_seed_to_seed_32cubed": rel_l2(coarse(Fr), coarse(Fs)),
        "absorbed_fraction": {k: [float(x) / n for x in outs[k]["absorbed"]] for k in outs},
        "error_vs_oracle": {"sdf": prefix_error(smcrt, desc, seed, 20000, precision),
                            "voxel": prefix_error(smcrt, desc, seed, 20000, precision, geometry="voxel")},
    })
    return res


def paper_speed_tests(smcrt, workloads, precision):
    """The paper's speed experiments (Sec. 3.2) on this GPU, both geometry
    models, whole runs timed (tables, voxelisation, walk):
    - tally-free speed test: isotropic scattering sphere (r = 0.5 cm, source
      at the centre) at radial optical depths 0.1, 1, 10, 100; 1e7 photons;
      no fluence tally (the voxel model walks a 200^3 grid);
    - Table 2, Jacques slab: the 420 nm medium of Table 1 (mu_a 1.8, mu_s'
      82 /cm, g 0.9, n 1.38) as a 2 x 2 x 4 cm slab under uniform normal
      illumination of its top face, 200 x 200 x 400 grid, 1e7 photons;
    - Table 2, isotropic sphere: tau = 100 with a 200^3 grid, 1e6 photons.
    The paper's CPU timings (Table 2) are returned beside them as context."""
    import torch
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))["table2_timings_cpu"]

    def timed(desc, n, geometry, tally, seed=1):
        eng = smcrt.Engine(0, precision=precision)
        sc = smcrt.Scene(dict(desc, geometry=geometry))
        smcrt.launch(eng, sc, seed + 1000, min(n, 200_000), outputs=smcrt.Outputs(sc, tally=tally))  # warm-up
        out = smcrt.Outputs(sc, tally=tally)
        torch.cuda.synchronize()
        t = time.perf_counter()
        smcrt.launch(eng, sc, seed, n, outputs=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        h = out.host()
        eng.close()
        return dt, h["interactions"] / n

    sweep = []
    for tau in (0.1, 1.0, 10.0, 100.0):
        desc = workloads.with_grid(workloads.scattering_sphere(tau), [200] * 3, lo=[-0.5] * 3, hi=[0.5] * 3)
        ts, ns = timed(desc, 10_000_000, "sdf", False)
        tv, nv = timed(desc, 10_000_000, "voxel", False)
        sweep.append({"tau": tau, "sdf_s": ts, "voxel_s": tv, "sdf_over_voxel_speed": tv / ts,
                      "mean_scatterings": ns, "eq4": tau * tau / 2 + tau,
                      "error_vs_oracle": prefix_error(smcrt, desc, 1, 20000 if tau < 50 else 2000, precision)})
    slab = workloads.semi_infinite_slab(1.8, 82.0, half_xy=1.0, nz=400)
    slab = workloads.with_grid(slab, [200, 200, 400], lo=[-1.0, -1.0, -4.0], hi=[1.0, 1.0, 0.0])
    slab["source"] = {"kind": "rect", "c": [0.0, 0.0, 0.5 * slab["pad"]], "half": [1.0, 1.0], "u": [0.0, 0.0, -1.0]}
    sphere = workloads.with_grid(workloads.scattering_sphere(100.0), [200] * 3, lo=[-0.5] * 3, hi=[0.5] * 3)
    table2 = {}
    for name, desc, n in (("jacques_slab", slab, 10_000_000), ("isotropic_sphere", sphere, 1_000_000)):
        ts, _ = timed(desc, n, "sdf", True)
        tv, _ = timed(desc, n, "voxel", True)
        g = gold[name]
        table2[name] = {"photons": n, "grid": g["grid"], "sdf_s": ts, "voxel_s": tv, "sdf_over_voxel_speed": tv / ts,
                        "paper_cpu_sdf_s": g["smcrt_s"], "paper_cpu_voxel_s": g["voxel_s"],
                        "paper_sdf_over_voxel_speed": g["voxel_s"] / g["smcrt_s"]}
    table2["context_only"] = True  # the paper's CPU timings beside ours: context, not a measured target
    return {"tally_free_sphere": sweep, "table2": table2}


def batching(smcrt, workloads, precision):
    """Batched persistent launches against the plain one-scene-per-launch
    walk on the same jobs (identical packets and results, so equal fluence
    error):
    - the small sphere case at its full 1e5 packets, 64 times (seeds differ);
    - the batched microvascular network at its stated size: 64 vessel
      networks (2000 capsules through the uniform grid, 128^3 grids, mu_s
      scaled 0.5-2x), 1e7 packets each, in ONE launch whose launch options
      the engine's autotuner picks on a batched launch of 16 of the scenes
      at 5e5 packets each (both forms then run with them); one scene per
      launch timed on 8 of them; the error
      against the oracle on 4 of the scenes (1e4 packets each, run as one
      batch)."""
    import numpy as np
    import torch

    from oracle import oracle as orc
    res = {}
    # small sphere x 64
    descs, n = [workloads.sphere_scene()] * 64, 100_000
    eng = smcrt.Engine(0, precision=precision)
    scenes = [smcrt.Scene(d) for d in descs]
    seeds = list(range(64))
    smcrt.launch_batch(eng, scenes, seeds, [20_000] * 64)  # warm-up
    outs = [smcrt.Outputs(sc) for sc in scenes]
    torch.cuda.synchronize()
    t = time.perf_counter()
    smcrt.launch_batch(eng, scenes, seeds, [n] * 64, outputs=outs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    outs = [smcrt.Outputs(sc) for sc in scenes]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for sc, sd, o in zip(scenes, seeds, outs):
        smcrt.launch(eng, sc, sd, n, outputs=o)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    res["sphere_1e5_x64"] = {"jobs": 64, "packets_per_job": n, "batched_packets_per_s": 64 * n / t_batch,
                             "one_per_launch_packets_per_s": 64 * n / t_plain, "speedup": t_plain / t_batch,
                             "error_vs_oracle": prefix_error(smcrt, descs[0], 0, 20000, precision, engine=eng)}
    eng.close()
    del outs
    # microvascular networks: 64 x 1e7
    descs = workloads.vessel_batch(64, n_caps=2000, n_grid=128)
    n = 10_000_000
    eng = smcrt.Engine(0, precision=precision)
    scenes = [smcrt.Scene(d) for d in descs]
    seeds = [5000 + i for i in range(64)]
    default_opts = eng.opts()
    # timed on a batch of 16 of the scenes at 5e5 packets each: long enough
    # that the launch is not its tail, two scenes per XCD as in the full batch
    _, tuned_rate = eng.autotune(scenes[:16], n_trial=500_000)
    smcrt.launch_batch(eng, scenes, seeds, [20_000] * 64)  # warm-up (tables, grids, code)
    outs = [smcrt.Outputs(sc) for sc in scenes]
    torch.cuda.synchronize()
    t = time.perf_counter()
    smcrt.launch_batch(eng, scenes, seeds, [n] * 64, outputs=outs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    hs = [o.host() for o in outs]
    del outs
    per = {k: sum(h[k] for h in hs) / (64 * n) for k in ("steps", "interactions", "interfaces", "voxel_pieces")}
    identity = max(abs(h["absorbed"].sum() + h["escaped_face"].sum() + h["roulette_loss"] - h["roulette_gain"]
                       + h["stalled"] - h["launched"]) / h["launched"] for h in hs)
    outs = [smcrt.Outputs(sc) for sc in scenes[:8]]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for sc, sd, o in zip(scenes[:8], seeds[:8], outs):
        smcrt.launch(eng, sc, sd, n, outputs=o)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    del outs
    # error against the oracle: 4 scenes, packets [0, 1e4) of their seeds, one batch
    m = 10_000
    g = smcrt.run_batch(descs[:4], seeds[:4], [m] * 4, engine=eng, precision=precision)
    errs = []
    for d, sd, gi in zip(descs[:4], seeds[:4], g):
        o = orc.run(d, sd, m)
        errs.append({"packets": m,
                     "fluence_relative_l2": float(np.linalg.norm(gi["fluence_raw"] - o["fluence_raw"])
                                                  / np.linalg.norm(o["fluence_raw"])),
                     "absorbed_relative": float(abs(gi["absorbed"].sum() - o["absorbed"].sum()) / o["absorbed"].sum())})
    res["vessels_1e7_x64"] = {
        "workload": "64 vessel networks (2000 capsules, radii 5-50 um, 2 mm cube), 128^3 grids, 1e7 packets each",
        "jobs": 64, "packets_per_job": n, "batched_packets_per_s": 64 * n / t_batch, "batched_s": t_batch,
        "one_per_launch_packets_per_s": 8 * n / t_plain, "one_per_launch_jobs_timed": 8,
        "speedup": (64 * n / t_batch) / (8 * n / t_plain), "per_packet": per,
        "energy_identity_residual_max": identity, "error_vs_oracle": errs, "launch": eng.opts(),
        "launch_default": default_opts, "autotune_trial_packets_per_s": tuned_rate}
    eng.close()
    return res


def csg_scenes(smcrt, workloads, precision, n=10_000_000):
    """Packets/s of the SDF walk on the two CSG scenes: the
    glass sphere under a beam in a scattering medium and the partly filled
    glass bottle (intersection and difference regions), 64^3 grids."""
    import torch
    res = {}
    for name in ("glass_sphere", "bottle"):
        desc = workloads.WORKLOADS[name](n_grid=64)
        eng = smcrt.Engine(0, precision=precision)
        sc = smcrt.Scene(desc)
        smcrt.launch(eng, sc, 77, 500_000, outputs=smcrt.Outputs(sc))  # warm-up
        out = smcrt.Outputs(sc)
        torch.cuda.synchronize()
        t = time.perf_counter()
        smcrt.launch(eng, sc, 1, n, outputs=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        h = out.host()
        res[name] = {"packets": n, "packets_per_s": n / dt, "steps_per_packet": h["steps"] / n,
                     "interfaces_per_packet": h["interfaces"] / n, "interactions_per_packet": h["interactions"] / n,
                     "error_vs_oracle": prefix_error(smcrt, desc, 1, 20000, precision, engine=eng)}
        eng.close()
    return res


def escape_images(smcrt, workloads, precision, n=10_000_000):
    """Single-plane output (Sec. 5): diffuse reflectance image of the Table 1
    420 nm slab (2 x 2 x 4 cm, uniform normal illumination of its top face)
    on a 200 x 200 pixel detector over the top face, with no fluence grid and
    with the 200 x 200 x 400 grid beside it; 1e7 photons, whole runs timed."""
    import torch
    slab = workloads.semi_infinite_slab(1.8, 82.0, half_xy=1.0, nz=400)
    slab = workloads.with_grid(slab, [200, 200, 400], lo=[-1.0, -1.0, -4.0], hi=[1.0, 1.0, 0.0])
    slab["source"] = {"kind": "rect", "c": [0.0, 0.0, 0.5 * slab["pad"]], "half": [1.0, 1.0], "u": [0.0, 0.0, -1.0]}
    slab["detector"] = {"face": 5, "lo": [-1.0, -1.0], "hi": [1.0, 1.0], "dims": [200, 200]}
    res = {}
    for name, tally in (("image_only", False), ("image_and_fluence", True)):
        eng = smcrt.Engine(0, precision=precision)
        sc = smcrt.Scene(slab)
        smcrt.launch(eng, sc, 99, 200_000, outputs=smcrt.Outputs(sc, tally=tally))  # warm-up
        out = smcrt.Outputs(sc, tally=tally)
        torch.cuda.synchronize()
        t = time.perf_counter()
        smcrt.launch(eng, sc, 1, n, outputs=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        h = out.host()
        res[name] = {"packets": n, "packets_per_s": n / dt,
                     "diffuse_reflectance": float(h["image"].sum()) / n,
                     "top_face_escape": float(h["escaped_face"][5]) / n}
        if tally:
            res[name]["error_vs_oracle"] = prefix_error(smcrt, slab, 1, 20000, precision, engine=eng)
        eng.close()
    return res


def step_shortcuts(smcrt, workloads, precision, omega=1.9):
    """The two step shortcuts of Sec. 5 against plain steps on the same
    packets -- over-relaxed sphere tracing (omega) and segment-traced steps
    (tangent bounds of convex shapes) -- : packets/s and sphere-tracing
    steps per packet of the layered slab (200^3 grid, 2e6 packets), the
    vessel cylinder (256^3, 2e6), the glass sphere and the bottle (64^3, 4e6
    each) and the 2000-capsule vessel network (128^3, 4e6); each shortcut's
    walk against the oracle's plain march on 1e4 of the same packets."""
    import torch
    res = {}
    cases = (("slab", 200, 2_000_000), ("cylinder", 256, 2_000_000), ("glass_sphere", 64, 4_000_000),
             ("bottle", 64, 4_000_000), ("vessels", 128, 4_000_000))
    for name, n_grid, n in cases:
        progress(f"step shortcuts: {name}")
        if name == "vessels":
            base = workloads.vessel_scene(3, 1.0, n_caps=2000, n_grid=n_grid)
        else:
            base = workloads.WORKLOADS[name](n_grid=n_grid)
        row = {"packets": n}
        for mode, extra in (("plain", {}), ("relaxed", {"relax": omega}), ("segment", {"segment": True})):
            desc = dict(base, **extra)
            eng = smcrt.Engine(0, precision=precision)
            sc = smcrt.Scene(desc)
            smcrt.launch(eng, sc, 77, min(n, 200_000), outputs=smcrt.Outputs(sc))  # warm-up
            out = smcrt.Outputs(sc)
            torch.cuda.synchronize()
            t = time.perf_counter()
            smcrt.launch(eng, sc, 1, n, outputs=out)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            h = out.host()
            row[mode] = {"packets_per_s": n / dt, "steps_per_packet": h["steps"] / n}
            eng.close()
            if mode != "plain":
                row[mode]["speedup"] = row[mode]["packets_per_s"] / row["plain"]["packets_per_s"]
                # the shortcut's walk against the oracle's plain march on the same packets
                row[mode]["error_vs_oracle"] = prefix_error(smcrt, desc, 1, 2000 if name == "vessels" else 10000,
                                                            precision, oracle_desc=base)
        row["omega"] = omega
        res[name] = row
    return res


def copy_calibration(smcrt, desc, steps):
    import torch
    sc = smcrt.Scene(desc)
    n = sc.n_voxels
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()
    ptr = smcrt._stream_ptr(st)
    smcrt.smcrt_normalize_fluence(sc.h, smcrt.C.c_void_p(src.data_ptr()), 1.0, smcrt.C.c_void_p(dst.data_ptr()), ptr)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(st)
    for _ in range(steps):
        smcrt.smcrt_normalize_fluence(sc.h, smcrt.C.c_void_p(src.data_ptr()), 1.0, smcrt.C.c_void_p(dst.data_ptr()), ptr)
    b.record(st)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    print(json.dumps({"copy_calibration": {"bytes_read": 8 * n, "bytes_written": 8 * n, "ms": ms,
                                           "GB/s": 16 * n / (ms * 1e-3) / 1e9, "launches": steps + 1}}))


def vessel_profile(smcrt, workloads, n_scenes, n, steps, warmup, precision):
    """The batched microvascular network alone (for profiling): n_scenes
    vessel scenes (2000 capsules each through the uniform grid, 128^3 grids,
    mu_s scaled 0.5-2x) in one persistent launch, n packets per scene per
    step; one JSON line with packets/s, kernel time per launch and the work
    counters per packet."""
    import numpy as np
    import torch
    descs = workloads.vessel_batch(n_scenes, n_caps=2000, n_grid=128)
    eng = smcrt.Engine(0, precision=precision)
    scenes = [smcrt.Scene(d) for d in descs]
    outs = [smcrt.Outputs(sc) for sc in scenes]
    st = torch.cuda.current_stream()
    for w in range(warmup):
        smcrt.launch_batch(eng, scenes, [900 + w] * n_scenes, [n] * n_scenes, outputs=outs, stream=st)
    torch.cuda.synchronize()
    for o in outs:
        o.zero_()
    marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        marks[k][0].record(st)
        smcrt.launch_batch(eng, scenes, [k * n_scenes + i for i in range(n_scenes)], [n] * n_scenes, outputs=outs,
                           stream=st)
        marks[k][1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    hs = [o.host() for o in outs]
    tot = {k: sum(h[k] for h in hs) for k in ("launched", "steps", "interactions", "interfaces", "voxel_pieces")}
    print(json.dumps({"vessel_batch": {
        "scenes": n_scenes, "packets_per_scene": n, "precision": precision, "steps": steps,
        "packets_per_s": n * n_scenes * steps / wall,
        "launch_ms": float(np.mean([a.elapsed_time(b) for a, b in marks])),
        "per_packet": {k: tot[k] / tot["launched"] for k in ("steps", "interactions", "interfaces", "voxel_pieces")},
        "launch": eng.opts()}}))
    eng.close()


def scene_profile(smcrt, workloads, name, n, steps, warmup, precision):
    """One workload family alone (for profiling): the scene at its stated
    grid, n packets per launch on one engine with default options; one JSON
    line with packets/s, kernel time per launch and the work counters per
    packet."""
    import numpy as np
    import torch
    desc = workloads.WORKLOADS[name]()
    eng = smcrt.Engine(0, precision=precision)
    sc = smcrt.Scene(desc)
    out = smcrt.Outputs(sc)
    st = torch.cuda.current_stream()
    for w in range(warmup):
        smcrt.launch(eng, sc, 900 + w, n, outputs=out, stream=st)
    torch.cuda.synchronize()
    out.zero_()
    marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        marks[k][0].record(st)
        smcrt.launch(eng, sc, k, n, outputs=out, stream=st)
        marks[k][1].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    h = out.host()
    print(json.dumps({"scene_profile": {
        "scene": name, "grid": desc["grid"]["dims"], "packets": n, "precision": precision, "steps": steps,
        "packets_per_s": n * steps / wall,
        "launch_ms": [round(a.elapsed_time(b), 2) for a, b in marks],
        "per_packet": {k: h[k] / h["launched"] for k in ("steps", "interactions", "interfaces", "voxel_pieces",
                                                         "grid_atomics")},
        "launch": eng.opts()}}))
    eng.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--packets", type=float, default=1e7)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle, comparator and serving legs (profiling runs)")
    ap.add_argument("--no-comparator", action="store_true",
                    help="skip the voxel-vs-SDF geometry comparison and the paper's speed experiments")
    ap.add_argument("--serve-requests", type=int, default=200, help="requests in the serving leg (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=0.0,
                    help="Poisson arrival rate of the serving leg (1/s); 0 = 70%% of the measured capacity")
    ap.add_argument("--serve-max-packets", type=float, default=1e6, help="largest request of the serving leg")
    ap.add_argument("--serve-budget", type=float, default=float(SERVE_BUDGET),
                    help="HBM budget of the serving leg's server in bytes")
    ap.add_argument("--serve-only", action="store_true",
                    help="only run the serving leg and print its JSON line (for the full request stream)")
    ap.add_argument("--vessels", type=int, default=0,
                    help="only run the batched vessel networks: this many scenes, --packets per scene per step")
    ap.add_argument("--scene", default="",
                    help="only run this workload family (sphere, cylinder, glass_sphere, ...) at its stated grid, "
                         "--packets per launch, and print its JSON line (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only stream the 200^3 FP64 grid through the fluence normalisation kernel "
                         "(a plain read-once/write-once copy of known size) and report its bandwidth")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2112_08035_amd import smcrt, workloads

    if args.serve_only:
        print(json.dumps({"serving": serving(smcrt, workloads, args.serve_requests, args.serve_rate,
                                             args.serve_max_packets, args.precision, budget=int(args.serve_budget))}))
        return
    if args.scene:
        scene_profile(smcrt, workloads, args.scene, int(args.packets), args.steps, args.warmup, args.precision)
        return
    if args.vessels > 0:
        vessel_profile(smcrt, workloads, args.vessels, int(args.packets), args.steps, args.warmup, args.precision)
        return
    desc = workloads.slab_scene()
    if args.copy_calibration:
        copy_calibration(smcrt, desc, args.steps)
        return
    n = int(args.packets)
    eng = smcrt.Engine(0, precision=args.precision)
    sc = smcrt.Scene(desc)
    out = smcrt.Outputs(sc)
    stream = torch.cuda.current_stream()

    for w in range(args.warmup):
        smcrt.launch(eng, sc, 900 + w, n, outputs=out, stream=stream)
    torch.cuda.synchronize()
    out.zero_()
    torch.cuda.synchronize()

    marks = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        marks[k][0].record(stream)
        smcrt.launch(eng, sc, k, n, outputs=out, stream=stream)
        marks[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [a.elapsed_time(b) for a, b in marks]
    launch_ms = float(np.mean(step_ms))
    h = out.host()
    steps = args.steps
    value = n * steps / wall
    per = {k: h[k] / steps for k in ("launched", "steps", "interactions", "interfaces", "advances",
                                      "voxel_pieces", "grid_atomics")}
    lane_ops = slab_lane_ops(per, len(desc["prims"]))
    achieved = lane_ops / (launch_ms * 1e-3)
    ceiling = atomic_ceiling()
    counters = measured_counters() if args.precision == "f32" else {}
    reqs = counters.get("atomic_requests_per_launch")
    identity = (h["absorbed"].sum() + h["escaped_face"].sum() + h["roulette_loss"] - h["roulette_gain"]
                + h["stalled"] - h["launched"])

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": "layered slab, 3 boxes 2x2 cm (0.01/0.2/1 cm), pencil beam, 1e7 packets/step, 200^3 FP64 fluence grid",
            "packets_per_step": n,
            "grid": [200, 200, 200],
            "transport": args.precision,
            "tallies": "f64",
            "launch": eng.opts(),
        },
        "per_packet": {k: per[k] / n for k in ("steps", "interactions", "interfaces", "voxel_pieces", "grid_atomics")},
        "energy_identity_residual": identity / h["launched"],
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "Tlane-op/s",
            "frac": achieved / PEAK_LANE_OPS,
            "frac_coarse_interface_price": slab_lane_ops(per, len(desc["prims"]), True) / (launch_ms * 1e-3)
            / PEAK_LANE_OPS,
            "traffic": counters.get("traffic_bytes_per_launch"),
            "kernel_ms": launch_ms,
            "step_kernel_ms": step_ms,
            "lane_ops_per_launch": lane_ops,
            "grid_atomics_per_s": per["grid_atomics"] / (launch_ms * 1e-3),
            "atomic_requests_per_launch": reqs,
            "atomic_request_ceiling_per_s": ceiling,
            "atomic_request_frac": (reqs / (launch_ms * 1e-3) / ceiling) if (ceiling and reqs) else None,
        },
    }

    if not args.no_cpu:
        from oracle import oracle as orc
        # the oracle's OpenMP team: OMP_NUM_THREADS when set, else the CPUs
        # this process may run on
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or avail
        cpu_model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                          if ln.startswith("model name")), "unknown") if os.path.exists("/proc/cpuinfo") else "unknown"
        # calibrate on a run long enough to hide the per-thread grid set-up,
        # then time a sample of about cpu_seconds
        # time = fixed set-up (per-thread grids) + packets / rate: fit both
        # from two short runs, then size the sample to about cpu_seconds
        tt = []
        for m in (20000, 80000):
            t = time.perf_counter()
            orc.run(desc, 0, m)
            tt.append(time.perf_counter() - t)
        rate0 = 60000 / max(tt[1] - tt[0], 1e-3)
        setup = max(tt[0] - 20000 / rate0, 0.0)
        n_cpu = int(max(20000, min(5_000_000, rate0 * max(args.cpu_seconds - setup, 1.0))) // 1000 * 1000)
        t = time.perf_counter()
        o = orc.run(desc, 0, n_cpu)
        cpu_s = time.perf_counter() - t
        # the same oracle on one thread, on a sample of about 4 s
        n_one = int(max(2000, min(n_cpu, 4.0 * n_cpu / cpu_s / threads)) // 1000 * 1000)
        t = time.perf_counter()
        orc.run(desc, 0, n_one, threads=1)
        one_s = time.perf_counter() - t
        result["cpu_baseline"] = {
            "value": n_cpu / cpu_s,
            "unit": "packets/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"packets [0, {n_cpu}) of the same slab workload, seed 0, FP64 oracle, {cpu_s:.1f} s",
            "one_thread_value": n_one / one_s,
            "one_thread_sample": f"packets [0, {n_one}), {one_s:.1f} s",
            "cpu_model": cpu_model,
            "cpus_available": avail,
        }
        # fluence error of the GPU path on the same packets
        g = smcrt.run(sc, 0, n_cpu, engine=eng, precision=args.precision)
        Fo, Fg = o["fluence_raw"], g["fluence_raw"]
        result["fluence_error"] = {
            "packets": n_cpu,
            "relative_l2": float(np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo)),
            "absorbed_relative": float(abs(g["absorbed"].sum() - o["absorbed"].sum()) / o["absorbed"].sum()),
            "z_scores": fluence_z_scores(smcrt, sc, eng, args.precision, desc, n_cpu, Fo),
        }
        result["trace_parity"] = trace_parity(smcrt, workloads, args.precision)
        progress("headline, oracle baseline and trace parity done")
    if not args.no_cpu and not args.no_comparator:
        result["voxel_comparator"] = comparator(smcrt, workloads, args.precision)
        progress("voxel comparator done")
        result["paper_speed_tests"] = paper_speed_tests(smcrt, workloads, args.precision)
        progress("paper speed tests done")
        result["csg_scenes"] = csg_scenes(smcrt, workloads, args.precision)
        result["batching"] = batching(smcrt, workloads, args.precision)
        progress("batching done")
        result["escape_images"] = escape_images(smcrt, workloads, args.precision)
        result["step_shortcuts"] = step_shortcuts(smcrt, workloads, args.precision)
        progress("escape images and step shortcuts done")
    if args.serve_requests > 0 and not args.no_cpu:
        result["serving"] = serving(smcrt, workloads, args.serve_requests, args.serve_rate,
                                    args.serve_max_packets, args.precision)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
