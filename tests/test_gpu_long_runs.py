"""Full-length parity of the benchmark channels against stored oracle runs.

The references under tests/golden/long_*.npz were written by
tests/golden/make_long_runs.py, which calls only the FP64 oracle: the
diagnostics (Sigma phi, Sigma psi, phi-weighted centroid and velocity, p_in,
p_out, extrema) every 100 (500) steps and, at the last step, phi, p, ux, uy,
T, psi on a strided sub-lattice plus the full row and column through the
initial bubble centre.

Over these horizons the method itself is ill-conditioned: the same FP64
kernel with its initial populations changed by one ulp drifts from itself by
~1e-4 (phi, u) after 2000 steps and by ~1e-2 after 20000 on the 1024x512
channels, while integral quantities stay put (the centroid to ~1e-5 lattice
units).  So the fields are compared against that sensitivity, measured in
the same test on the GPU (FP64, one-ulp perturbation of every initial
population): each field's max-rel against the oracle must stay within three
times the perturbation's own max-rel, and the centroid within a fixed bar.

  * The four 1024x512 FP32 channels (NF and SRF at beta_s 0 and 0.2), 20000
    steps in one batched handle: centroid within 1e-3 lattice units of the
    oracle's at every logged step (100 steps apart); phi, T, psi and u (as a
    vector) within the sensitivity bar, for FP32 and FP64 alike.
  * The 2048x1024 channel, 10000 steps, in FP16 storage, FP32 and FP64: FP16
    storage keeps the centroid within 0.05 lattice units at every logged step
    and the pressure jump p_in - p_out within 1 %; FP32 and FP64 keep the
    centroid within 1e-3 lattice units and the fields within the sensitivity
    bar.  The table of per-field max-rel, drift of Sigma phi and Sigma psi,
    and centroid error of the three storage forms is printed.
  * The 64 seeded uneven FP32 channels in one handle over their 5000 steps:
    every case bitwise equal to the same case run alone in the same
    configuration; the smallest (256x128) against its stored oracle run
    (centroid within 1e-3 lattice units at every 100th step, fields at the
    end within three times the rounding spread, see check_against_stored).
  * The 4096x2048 FP16-storage channel beside 256 seeded 128x64 FP32
    channels, with budgets of 5000 and 2000 steps: the budgets hold, the
    large case and every 32nd small one are bitwise equal to separate runs,
    the first small one matches its stored oracle run, and the large case
    keeps its centroid within 0.05 lattice units and p_in - p_out within 1 %
    of the same case in the FP64 mode after 5000 steps.
"""
import hashlib
import os

import numpy as np
import pytest

from paper_2408_00146_amd import cases

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")
FIELDS = ("phi", "p", "ux", "uy", "T", "psi")


def oracle_sha() -> str:
    h = hashlib.sha256()
    for name in ("lbm_oracle.c", "lbm_oracle.h"):
        with open(os.path.join(ROOT, "oracle", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load(name):
    path = os.path.join(GOLD, f"long_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} has not been written (tests/golden/make_long_runs.py)")
    z = np.load(path)
    assert str(z["oracle_sha256"]) == oracle_sha(), "reference written by another oracle source: regenerate it"
    return z


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_00146_amd import lbm as L

    L.lib()
    return L


def sample(f, z, p):
    """The GPU fields on the stored nodes: strided sub-lattice, row, column."""
    st = int(z["stride"])
    out = {}
    for k in FIELDS:
        a = np.asarray(f[k])
        out[k] = np.concatenate([a[::st, ::st].ravel(), a[int(z["row_y"]), :], a[:, int(z["col_x"])]])
    return out


def stored(z, prefix=""):
    out = {}
    for i, k in enumerate(FIELDS):
        out[k] = np.concatenate([z[prefix + "fields"][i].ravel(), z[prefix + "row"][i], z[prefix + "col"][i]])
    return out


def errors(g, r):
    e = {k: float(np.max(np.abs(g[k] - r[k])) / np.max(np.abs(r[k]))) for k in ("phi", "T", "psi")}
    e["u"] = float(np.max(np.hypot(g["ux"] - r["ux"], g["uy"] - r["uy"])) / np.max(np.hypot(r["ux"], r["uy"])))
    return e


def run_logged(s, ncases, steps, every):
    """Advance a handle, reducing each case every `every` steps (step 0 first)."""
    logs = [[s.reduce(i)] for i in range(ncases)]
    for _ in range(steps // every):
        s.step(every)
        for i in range(ncases):
            logs[i].append(s.reduce(i))
    return logs


def perturbed(s, ncases, seed=7, rel=2.0 ** -53):
    """Change every population of every case by `rel` of itself (random sign):
    one FP64 ulp by default, 2**-24 for one FP32 ulp."""
    rng = np.random.default_rng(seed)
    for i in range(ncases):
        P = s.populations(i)
        s.set_populations(P * (1 + rng.choice([-1.0, 1.0], size=P.shape) * rel), i)


def test_fp32_channels_20000_steps(lbm):
    ps = cases.config_fp32_runs()
    refs = {p["label"]: load(f"fp32_runs_{p['label']}") for p in ps
            if os.path.exists(os.path.join(GOLD, f"long_fp32_runs_{p['label']}.npz"))}
    if not refs:
        pytest.skip("no 1024x512 reference has been written")
    s32 = lbm.Solver(ps)
    logs = run_logged(s32, len(ps), 20000, 100)
    p64 = [dict(p, precision=cases.FP64) for p in ps]
    s64, s64p = lbm.Solver(p64), lbm.Solver(p64)
    perturbed(s64p, len(ps))
    s64.step(20000)
    s64p.step(20000)
    z0 = next(iter(refs.values()))
    names = list(z0["diag_names"])
    ix, iy = names.index("xc"), names.index("yc")
    for i, p in enumerate(ps):
        if p["label"] not in refs:
            continue
        z = refs[p["label"]]
        assert list(z["diag_steps"]) == list(range(0, 20001, 100))
        dx = max(max(abs(d["xc"] - r[ix]), abs(d["yc"] - r[iy])) for d, r in zip(logs[i], z["diag"]))
        ref = stored(z)
        g64 = sample(s64.fields(i), z, p)
        sens = errors(sample(s64p.fields(i), z, p), g64)
        e32 = errors(sample(s32.fields(i), z, p), ref)
        e64 = errors(g64, ref)
        print(p["label"], "max centroid error", dx, "FP32", e32, "FP64", e64, "one-ulp sensitivity", sens)
        assert dx <= 1e-3, (p["label"], dx)
        for k in ("phi", "T", "psi", "u"):
            assert e32[k] <= 3 * sens[k] and e64[k] <= 3 * sens[k], (p["label"], k, e32, e64, sens)


def test_precision_forms_2048x1024_10000_steps(lbm):
    z = load("precision_2048x1024")
    names = list(z["diag_names"])
    col = {k: names.index(k) for k in ("mass_phi", "mass_psi", "xc", "yc", "p_in", "p_out")}
    ref = stored(z)
    rd = z["diag"]
    table, fields = {}, {}
    for prec in (cases.FP16S, cases.FP32, cases.FP64, "FP64+ulp"):
        p = cases.config_precision(cases.FP64 if prec == "FP64+ulp" else prec)
        s = lbm.Solver(p)
        if prec == "FP64+ulp":
            perturbed(s, 1)
        log = run_logged(s, 1, 10000, 500)[0]
        fields[prec] = sample(s.fields(0), z, p)
        e = errors(fields[prec], ref)
        dc = max(np.hypot(d["xc"] - r[col["xc"]], d["yc"] - r[col["yc"]]) for d, r in zip(log, rd))
        dp_g = log[-1]["p_in"] - log[-1]["p_out"]
        dp_o = rd[-1][col["p_in"]] - rd[-1][col["p_out"]]
        drift = {k: abs(log[-1][k] - log[0][k]) / abs(log[0][k]) for k in ("mass_phi", "mass_psi")}
        table[prec] = dict(e, centroid=dc, dp_rel=abs(dp_g / dp_o - 1.0), **{f"drift_{k}": v for k, v in drift.items()})
        s.close()
    sens = errors(fields["FP64+ulp"], fields[cases.FP64])
    for prec, name in ((cases.FP16S, "FP16 storage"), (cases.FP32, "FP32"), (cases.FP64, "FP64")):
        print(name, {k: f"{v:.2e}" for k, v in table[prec].items()})
    print("FP64 one-ulp sensitivity", {k: f"{v:.2e}" for k, v in sens.items()})
    t16, t32, t64 = table[cases.FP16S], table[cases.FP32], table[cases.FP64]
    assert t16["centroid"] <= 0.05 and t16["dp_rel"] <= 0.01, t16
    for t in (t32, t64):
        assert t["centroid"] <= 1e-3, t
        assert all(t[k] <= 3 * sens[k] for k in ("phi", "T", "psi", "u")), (t, sens)


def check_against_stored(lbm, s, case, log, z, p, steps, fp32_floor=None):
    """Centroid at every logged step and end fields of one FP32 case of `s`
    against its stored oracle run.

    The field bars come from the rounding spread of the step itself, measured
    here and stored: configuration 0 (two nodes per thread, its own pull and
    operation order) evaluates the same step with other roundings, so its
    distance from the tested configuration, in FP32 and in the FP64 mode, is
    how far two valid evaluations drift apart on this case over this horizon;
    so are the FP64 mode started one ulp away, the oracle's own source built
    with FMA contraction (stored beside the reference), and in FP32 the
    tested configuration started one FP32 ulp away (two draws): where the
    flow is ill-conditioned, FP32 evaluations that differ only in rounding
    land on different branches (on the smallest seeded channel after 5000
    steps, 6e-5 to 2.3e-3 apart in phi).  FP64 must stay within three times
    the largest FP64 spread (at least 1e-12), FP32 within three times the
    largest FP32 spread (at least the FP32 bar of 1e-5, or the per-field
    floors given)."""
    names = list(z["diag_names"])
    ix, iy = names.index("xc"), names.index("yc")
    assert int(z["steps"]) == steps
    t = s.tile
    dx = max(max(abs(d["xc"] - r[ix]), abs(d["yc"] - r[iy])) for d, r in zip(log, z["diag"]))
    q32, q64 = dict(p, max_steps=0), dict(p, precision=cases.FP64, max_steps=0)
    runs = {}
    for name, q, cfg, ulp in (("fp32_cfg0", q32, 0, None), ("fp32_ulp1", q32, t, (1, 2.0 ** -24)),
                              ("fp32_ulp2", q32, t, (2, 2.0 ** -24)), ("fp64", q64, t, None),
                              ("fp64_cfg0", q64, 0, None), ("fp64_ulp", q64, t, (7, 2.0 ** -53))):
        with lbm.Solver(q) as r:
            r.set_tile(cfg)
            if ulp:
                perturbed(r, 1, seed=ulp[0], rel=ulp[1])
            r.step(steps)
            runs[name] = sample(r.fields(), z, p)
    g32 = sample(s.fields(case=case), z, p)
    ref = stored(z)
    e32, e64 = errors(g32, ref), errors(runs["fp64"], ref)
    s32 = [errors(runs[n], g32) for n in ("fp32_cfg0", "fp32_ulp1", "fp32_ulp2")]
    sp32 = {k: max(e[k] for e in s32) for k in s32[0]}
    a64, b64 = errors(runs["fp64_cfg0"], runs["fp64"]), errors(runs["fp64_ulp"], runs["fp64"])
    c64 = errors(stored(z, "spread_"), ref)
    sp64 = {k: max(a64[k], b64[k], c64[k]) for k in a64}
    print(p["label"], f"{steps} steps: centroid {dx:.2e}", "FP32", fmt(e32), "FP32 spread", fmt(sp32),
          "FP64", fmt(e64), "FP64 spread", fmt(sp64))
    assert dx <= 1e-3, dx
    for k in ("phi", "T", "psi", "u"):
        assert e64[k] <= max(1e-12, 3 * sp64[k]), (k, e64, sp64)
        assert e32[k] <= max((fp32_floor or {}).get(k, 1e-5), 3 * sp32[k]), (k, e32, sp32)


def fmt(e):
    return {k: f"{v:.2e}" for k, v in e.items()}


def test_batched64_5000_steps(lbm):
    ps = cases.config_batched()
    k = int(np.argmin([p["nx"] * p["ny"] for p in ps]))
    z = load(f"batched64_case{k}")
    s = lbm.Solver(ps)
    t = s.autotune(3)
    log = [s.reduce(k)]
    for _ in range(50):
        s.step(100)
        log.append(s.reduce(k))
    s.step(100)  # past every budget: nothing moves
    assert all(s.steps_done(i) == 5000 for i in range(len(ps)))
    for i, p in enumerate(ps):
        with lbm.Solver(p) as one:
            one.set_tile(t)
            one.step(5000)
            assert np.array_equal(one.populations(), s.populations(i)), i
    check_against_stored(lbm, s, k, log, z, ps[k], 5000)


def test_large_plus_small_full_budgets(lbm):
    ps = cases.config_large_plus_small()
    z = load("large_plus_small_case1")
    s = lbm.Solver(ps)
    t = s.autotune(3)
    log = [s.reduce(1)]
    for _ in range(50):
        s.step(100)
        log.append(s.reduce(1))
    assert s.steps_done(0) == 5000 and all(s.steps_done(i) == 2000 for i in range(1, len(ps)))
    for i in [0] + list(range(1, len(ps), 32)):
        with lbm.Solver(ps[i]) as one:
            one.set_tile(t)
            one.step(5000)
            assert np.array_equal(one.populations(), s.populations(i)), i
    # The velocity of this channel after 2000 steps is the decaying parasitic
    # current at the interface (max |u| 2.5e-4 at step 10, 2.2e-5 at step
    # 2000).  The FP32 error there stays near the rounding of the unit normal
    # and curvature (absolute 4e-11 after one step, 2.5e-10 after 2000, in
    # both FP32 configurations), so relative to the shrinking maximum it grows
    # from 4.7e-7 to 1.1e-5: the FP32 velocity bar is 2e-5 for this case.
    check_against_stored(lbm, s, 1, log[:21], z, ps[1], 2000, fp32_floor={"u": 2e-5})
    d16 = s.reduce(0)
    s.close()
    with lbm.Solver(dict(ps[0], precision=cases.FP64)) as a:
        a.step(5000)
        d64 = a.reduce()
    dc = float(np.hypot(d16["xc"] - d64["xc"], d16["yc"] - d64["yc"]))
    dp = abs((d16["p_in"] - d16["p_out"]) / (d64["p_in"] - d64["p_out"]) - 1.0)
    print("4096x2048 FP16 storage vs FP64 mode after 5000 steps: centroid", dc, "p_in - p_out", dp)
    assert dc <= 0.05 and dp <= 0.01, (dc, dp)
