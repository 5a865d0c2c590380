"""Comparison helpers for the GPU parity tests (no GPU needed to import)."""
import numpy as np


def mirror(desc, **kw):
    """The oracle's step-count mirror of the kernels' shortcuts (free-flight
    reuse and the ambient skip), for tests that compare numbers of SDF
    evaluations.  Its events and tallies are the plain march's (pinned in
    tests/test_oracle_mirror.py); every other comparison uses the plain
    march, the oracle's default."""
    return dict(desc, reuse=True, ambient_skip=True, **kw)


def extent_of(S, desc):
    """Largest side of the simulation volume the library uses for a scene."""
    sc = S.Scene(desc)
    _, _, lo, hi = S.smcrt_scene_info(sc.h)
    return float(np.max(hi - lo))


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
    interaction point.  The depth a record carries has been used up since
    the last time it was drawn (emission or scattering), in every medium
    crossed since, so its rounding error scales with the largest
    attenuation among those media (and the record's own): that one
    normalises it.  Where no medium has attenuated it yet, it is compared
    relative, floor 1.
    Returns (agreeing fraction, worst errors, list of (packet, record) of
    first disagreements)."""
    agree = 0
    worst = {"p": 0.0, "u": 0.0, "w": 0.0, "tau": 0.0}
    bad = []
    for pid, (o, g) in enumerate(zip(o_traces, g_traces)):
        o, g = o[:cap], g[:cap]
        ok = len(o) == len(g)
        m_seg = 0.0  # largest attenuation met since the depth was last drawn
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
            if a["type"] in ("EMIT", "SCATTER"):
                m_seg = 0.0
            if mut is not None and a["region"] >= 0:
                m_seg = max(m_seg, mut[a["region"]])
            m = m_seg
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


def diverged_fraction(o_traces, g_traces, cap=50):
    """Fraction of packets whose GPU walk takes another decision than the
    oracle's within the first cap records: an event whose type, region or
    index differs, or a different number of records.  Rounding alone
    (positions, directions) never counts; a flipped threshold decision
    (xi < R, s <= d, escape, region probe) does."""
    div = 0
    for o, g in zip(o_traces, g_traces):
        o, g = o[:cap], g[:cap]
        same = len(o) == len(g) and all((a["type"], a["region"], a["event"]) == (b["type"], b["region"], b["event"])
                                        for a, b in zip(o, g))
        div += not same
    return div / len(o_traces)


def batch_se(batches):
    """Standard error of the sum of independent batch tallies (per element)."""
    B = len(batches)
    arr = np.stack(batches)
    return np.sqrt(B * arr.var(axis=0, ddof=1))


# Scenes whose walks are chaotic billiards: long chains of reflections and
# total internal reflections on curved glass (the partly filled bottle, the
# scene of further shapes).  There the FP32 walk drifts from the FP64
# oracle's by rounding amplified at every curved hit (measured: 1e-6 cm
# after some 40 events, 4e-4 cm after 250), until a packet takes another
# decision -- about 2 packets in 1e4 on these scenes (bottle, seed 99:
# packets 9642 at event 44 and 8236 at event 255; shapes, seed 27: 7024 at
# event 81 and 7134 at event 139).  Such a packet is another valid walk and
# moves the absorbed total by at most its weight, <= 1.
CHAOTIC = ("bottle", "shapes")


def absorbed_agrees(g_total, o_total, n, prec, name=""):
    """Total absorbed weight of a run against the oracle's on the same
    packets: 1e-9 relative in FP64, 1e-4 in FP32; on the chaotic scenes in
    FP32, 1e-4 or at most 2 packets' weight per 1e4 packets."""
    diff = abs(g_total - o_total)
    rel = diff / abs(o_total)
    if prec == "f64":
        return rel <= 1e-9
    if name in CHAOTIC:
        return rel <= 1e-4 or diff <= 2.0 * n / 1e4
    return rel <= 1e-4


def identity_residual(r):
    return (r["absorbed"].sum() + r["escaped_face"].sum() + r["roulette_loss"] - r["roulette_gain"]
            + r["stalled"] - r["launched"])


def oracle_batches(orc, desc, seed, n, n_batches, voxel=False):
    """Oracle run of packets [0, n) in n_batches equal batches: summed
    tallies and the per-voxel standard error of the fluence sum."""
    step = n // n_batches
    outs = [orc.run(desc, seed, step, first=b * step, voxel=voxel) for b in range(n_batches)]
    tot = {k: sum(o[k] for o in outs) for k in ("absorbed", "escaped_face", "roulette_gain", "roulette_loss",
                                                "stalled", "launched", "interactions", "interfaces", "steps")}
    tot["fluence_raw"] = sum(o["fluence_raw"] for o in outs)
    se = batch_se([o["fluence_raw"] for o in outs])
    return tot, se


def voxel_diagonal(desc):
    g = desc["grid"]
    d = (np.array(g["hi"]) - np.array(g["lo"])) / np.array(g["dims"])
    return float(np.linalg.norm(d))


def check_fluence(g, o, se, desc, prec, frac_needed=0.995, n_batches=10):
    """Per voxel within 3 Monte Carlo SE (estimated from oracle batches).
    FP64: where no batch varies, the two must agree to rounding.  FP32: a
    packet whose FP32 walk flips a discrete decision becomes another valid
    walk; the voxels only it reaches have zero oracle variance, so the SE
    is floored at one packet's largest possible deposit (weight <= 1 times
    the voxel diagonal).  The grid's chi-square per degree of freedom --
    the mean squared z times (nu - 2)/nu, nu = n_batches - 1, which makes a
    Student-t z average 1 -- is at most 1.1: two independent samples would
    put it near 1, the same packets walked the same way near 0."""
    Fg, Fo = g["fluence_raw"], o["fluence_raw"]
    if prec == "f64":
        zero = se == 0
        assert np.all(np.abs(Fg[zero] - Fo[zero]) <= 1e-9 * Fo.max())
        sel = ~zero
        se_eff = se[sel]
    else:
        sel = (se > 0) | (Fg != Fo)
        se_eff = np.maximum(se[sel], voxel_diagonal(desc))
    z = np.abs(Fg[sel] - Fo[sel]) / se_eff
    within = np.mean(z <= 3.0)
    nu = n_batches - 1
    chi2 = float(np.mean(z ** 2)) * (nu - 2) / nu
    l2 = np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo)
    print(f"voxels within 3 SE: {within:.5f}, max z {z.max():.3f}, chi2/dof {chi2:.4f}, relative L2 {l2:.3e}")
    assert within >= frac_needed
    assert chi2 <= 1.1, chi2
    return l2


def independent_fluence_check(g_batches, o_batches, min_frac=0.99):
    """Statistical comparison of two INDEPENDENT samples of the fluence (the
    GPU on one packet-id range, the oracle on another), each given as B
    batch tallies of equal size.  Under the hypothesis that both walk the
    same distribution, the per-voxel variance of a batch is estimated from
    the two sets pooled (2B - 2 degrees of freedom) and the difference of
    the totals, divided by its estimated SE, is Student-t with nu = 2B - 2
    where the batch sums are Gaussian.  Voxels that every batch of both
    sets reaches are tested (elsewhere a few visits cannot be Gaussian):
    at least min_frac of them within 3 SE (t_38 puts 0.5 % beyond), and the
    grid's chi-square per degree of freedom -- the mean squared z times
    (nu - 2)/nu, the factor that makes it 1 in expectation under t -- in
    [0.9, 1.1].  Returns (fraction within 3 SE, chi2/dof, voxels tested)."""
    G, O = np.stack(g_batches), np.stack(o_batches)
    B = G.shape[0]
    assert O.shape[0] == B and B >= 10
    keep = np.all(G > 0, axis=0) & np.all(O > 0, axis=0)
    pooled = 0.5 * (G.var(axis=0, ddof=1) + O.var(axis=0, ddof=1))
    d = G.sum(axis=0) - O.sum(axis=0)
    z2 = d[keep] ** 2 / (2.0 * B * pooled[keep])
    nu = 2 * B - 2
    chi2 = float(z2.mean()) * (nu - 2) / nu
    within = float(np.mean(np.sqrt(z2) <= 3.0))
    print(f"independent samples: {int(keep.sum())} voxels, within 3 SE {within:.4f}, chi2/dof {chi2:.4f}")
    assert keep.sum() >= 2000, keep.sum()
    assert within >= min_frac
    assert 0.9 <= chi2 <= 1.1
    return within, chi2, int(keep.sum())
