"""Comparison helpers for the GPU parity tests (no GPU needed to import)."""
import numpy as np


def compare_traces(o_traces, g_traces, extent, tol, cap=50, mut=None):
    """Event-by-event comparison of oracle and GPU traces of the same
    packets.  A packet agrees when, for its first min(cap, length) records,
    event index, type and region are equal and position (relative to the
    scene extent), direction, weight and remaining optical depth (relative,
    floor 1) differ by at most tol.  Escape records are compared modulo
    sliding along the exit ray: the recorded point is the first
    sphere-tracing point beyond the volume, whose place on the ray depends
    on the step sequence, so the check is the GPU point's distance from the
    oracle's exit ray.  The remaining optical depth is compared as the
    remaining path tau/mu_t relative to the extent (mut: attenuation per
    region index, -1 = ambient), because that is what fixes the next
    interaction point; in ambient media it is compared relative, floor 1.
    Returns (agreeing fraction, worst errors, list of (packet, record) of
    first disagreements)."""
    agree = 0
    worst = {"p": 0.0, "u": 0.0, "w": 0.0, "tau": 0.0}
    bad = []
    for pid, (o, g) in enumerate(zip(o_traces, g_traces)):
        o, g = o[:cap], g[:cap]
        ok = len(o) == len(g)
        for i in range(min(len(o), len(g))):
            a, b = o[i], g[i]
            if (a["type"], a["region"], a["event"]) != (b["type"], b["region"], b["event"]):
                ok = False
                bad.append((pid, i, a["type"], b["type"]))
                break
            if a["type"] == "ESCAPE":
                d = b["p"] - a["p"]
                ep = np.linalg.norm(d - (d @ a["u"]) * a["u"]) / extent
            else:
                ep = np.max(np.abs(a["p"] - b["p"])) / extent
            errs = {"p": ep, "u": np.max(np.abs(a["u"] - b["u"])),
                    "w": abs(a["w"] - b["w"]) / max(abs(a["w"]), 1e-300),
                    "tau": abs(a["tau"] - b["tau"]) / max(1.0, abs(a["tau"]))}
            m = mut[a["region"]] if (mut is not None and a["region"] >= 0) else 0.0
            if m > 0:
                errs["tau"] = abs(a["tau"] - b["tau"]) / (m * extent)
            for k, v in errs.items():
                worst[k] = max(worst[k], v)
            if max(errs.values()) > tol:
                ok = False
                bad.append((pid, i, a["type"], b["type"]))
                break
        agree += ok
    return agree / len(o_traces), worst, bad


def batch_se(batches):
    """Standard error of the sum of independent batch tallies (per element)."""
    B = len(batches)
    arr = np.stack(batches)
    return np.sqrt(B * arr.var(axis=0, ddof=1))


def identity_residual(r):
    return (r["absorbed"].sum() + r["escaped_face"].sum() + r["roulette_loss"] - r["roulette_gain"]
            + r["stalled"] - r["launched"])
