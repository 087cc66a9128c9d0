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


def stored(z):
    out = {}
    for i, k in enumerate(FIELDS):
        out[k] = np.concatenate([z["fields"][i].ravel(), z["row"][i], z["col"][i]])
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


def perturbed(s, ncases, seed=7):
    """Change every population of every case by one ulp (random sign)."""
    rng = np.random.default_rng(seed)
    for i in range(ncases):
        P = s.populations(i)
        s.set_populations(P * (1 + rng.choice([-1.0, 1.0], size=P.shape) * 2.0 ** -53), i)


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
