"""CPU checks of the FSS post-processing (paper_1309_1599_amd.fss) on
synthetic runs whose xi_L/L curves are known lines through a common point."""
import numpy as np
import pytest

from paper_1309_1599_amd import fss


def _run(L, T, xi_over_L, n_samples, noise, seed, chi=10.0):
    """A run dict whose per-sample susceptibilities give xi/L = xi_over_L(T)
    and chi(0) = chi(T) in the disorder average (lattice Ornstein-Zernike
    form), with multiplicative sample noise."""
    rng = np.random.default_rng(seed)
    N = L ** 3
    chi0 = chi * (1 + noise * rng.normal(size=(n_samples, len(T))))
    xi = xi_over_L * L
    chik = chi0 / (1 + 4 * xi ** 2 * np.sin(np.pi / L) ** 2)
    q2 = np.stack([chi0 / N, chi0 / N * 1.01])          # last bin, then an earlier one
    qk2 = np.stack([chik / N, chik / N])
    return {"L": L, "temps": list(T), "n_samples": n_samples, "bins": [(5, 10), (2, 5)],
            "counts": [5, 3], "means": {"q2": q2.tolist(), "qk2": qk2.tolist(), "e": np.zeros_like(q2).tolist()}}


def test_crossing_nu_and_xi_at_the_crossing():
    T = np.linspace(0.8, 1.2, 12)
    Tc, yc, nu = 0.95, 0.6, 2.0
    s1 = -0.8                                    # d(xi_L/L)/dT
    # (d xi_2L/dT)/(d xi_L/dT) = 2^(1+1/nu)  =>  d(xi_2L/2L)/dT = s1 * 2^(1+1/nu) / 2
    s2 = s1 * 2 ** (1 + 1 / nu) / 2
    a = _run(8, T, yc + s1 * (T - Tc), 64, 0.0, 1)
    b = _run(16, T, yc + s2 * (T - Tc), 64, 0.0, 2)
    res = fss.analyse(a, b)
    assert res["T_cross"][0] == pytest.approx(Tc, abs=1e-9)
    assert res["xi_over_L_cross"][0] == pytest.approx(yc, abs=1e-9)
    assert res["nu"][0] == pytest.approx(nu, rel=1e-6)
    # with sample noise the estimate scatters within its jackknife error
    a = _run(8, T, yc + s1 * (T - Tc), 200, 0.02, 3)
    b = _run(16, T, yc + s2 * (T - Tc), 200, 0.02, 4)
    res = fss.analyse(a, b)
    assert abs(res["T_cross"][0] - Tc) < 5 * res["T_cross"][1] + 1e-3
    assert res["T_cross"][1] > 0


def test_xi_over_L_and_thermalisation():
    T = np.linspace(0.8, 1.2, 5)
    r = _run(8, T, np.full(5, 0.5), 16, 0.0, 5)
    xi, err = fss.xi_over_L(r)
    np.testing.assert_allclose(xi, 0.5, rtol=1e-12)
    th = fss.thermalisation(r)
    assert th[0]["diff"] == pytest.approx([0.0] * 5)
    assert np.allclose(th[1]["diff"], 0.01 * 10.0)   # the earlier bin was 1 % higher


def test_save_and_combine(tmp_path):
    """Two saved batches of independent samples combine into one run with
    the samples of both, and the analysis of the combination equals that of
    the concatenated runs."""
    T = np.linspace(0.8, 1.2, 12)
    Tc, yc, s1 = 0.95, 0.6, -0.8
    s2 = s1 * 2 ** 1.5 / 2
    batches = []
    for k in range(2):
        a = _run(8, T, yc + s1 * (T - Tc), 50, 0.02, 10 + k)
        b = _run(16, T, yc + s2 * (T - Tc), 50, 0.02, 20 + k)
        for r in (a, b):
            r.update(R=2, steps=100, measure_every=10, tau_walk=list(np.arange(50) * 0.5 + k))
            r["means"] = {key: np.asarray(v) for key, v in r["means"].items()}
        path = tmp_path / f"b{k}.npz"
        fss.save_runs(path, [a, b])
        batches.append((a, b, path))
    runs = fss.load_runs([str(p) for _, _, p in batches])
    assert [r["n_samples"] for r in runs] == [100, 100]
    both = [dict(batches[0][i], n_samples=100,
                 means={key: np.concatenate([batches[0][i]["means"][key], batches[1][i]["means"][key]], axis=1)
                        for key in ("q2", "qk2", "e")}) for i in (0, 1)]
    want = fss.analyse(*both)
    got = fss.analyse(*runs)
    assert got["T_cross"] == pytest.approx(want["T_cross"])
    # temperature-walk times travel with their samples: 0 .. 24.5 and 1 .. 25.5
    tau = np.concatenate([np.arange(50) * 0.5, np.arange(50) * 0.5 + 1])
    np.testing.assert_array_equal(runs[0]["tau_walk"], tau)
    w = fss.walk_summary(runs[0])
    assert w["max"] == 25.5 and w["median"] == pytest.approx(np.median(tau))
    assert w["runs_longer_than_10_tau"] == pytest.approx(np.mean(100 >= 10 * tau))


def test_chiral_channel():
    """The chiral-glass channel reads cg2 / cgk2 and finds its own crossing."""
    T = np.linspace(0.8, 1.2, 12)
    a = _run(8, T, 0.6 - 0.8 * (T - 0.95), 40, 0.0, 1)
    b = _run(16, T, 0.6 - 1.4 * (T - 0.95), 40, 0.0, 2)
    ac = _run(8, T, 0.05 - 0.1 * (T - 1.1), 40, 0.0, 3)
    bc = _run(16, T, 0.05 - 0.2 * (T - 1.1), 40, 0.0, 4)
    for r, c in ((a, ac), (b, bc)):
        r["means"]["cg2"] = c["means"]["q2"]
        r["means"]["cgk2"] = c["means"]["qk2"]
    assert fss.analyse(a, b)["T_cross"][0] == pytest.approx(0.95)
    res = fss.analyse(a, b, channel="cg")
    assert res["channel"] == "cg" and res["T_cross"][0] == pytest.approx(1.1)


@pytest.mark.parametrize("Ls,Ll", [(8, 16), (8, 12)])
def test_eta_and_nu_from_quotients(Ls, Ll):
    """chi_bL / chi_L = b^(2 - eta) and (d xi_bL/dT)/(d xi_L/dT) = b^(1 + 1/nu)
    at the crossing (Sec. IV), for the paper's b = 2 and for b = 3/2."""
    T = np.linspace(0.8, 1.2, 12)
    Tc, yc, nu, eta, s1 = 0.95, 0.6, 2.3, -0.4, -0.8
    b = Ll / Ls
    s2 = s1 * b ** (1 + 1 / nu) / b
    chi = 10.0 - 6.0 * (T - Tc)                        # linear: the local fits are exact
    a = _run(Ls, T, yc + s1 * (T - Tc), 32, 0.0, 1, chi=chi)
    c = _run(Ll, T, yc + s2 * (T - Tc), 32, 0.0, 2, chi=chi * b ** (2 - eta))
    res = fss.analyse(a, c)
    assert res["T_cross"][0] == pytest.approx(Tc, abs=1e-9)
    assert res["nu"][0] == pytest.approx(nu, rel=1e-6)
    assert res["eta"][0] == pytest.approx(eta, abs=1e-9)


def test_combine_from_the_command_line(tmp_path):
    """--combine analyses saved batches without a GPU and writes the report."""
    import json
    import os
    import subprocess
    import sys
    T = np.linspace(0.8, 1.2, 12)
    a = _run(8, T, 0.6 - 0.8 * (T - 0.95), 40, 0.01, 31)
    b = _run(16, T, 0.6 - 1.4 * (T - 0.95), 40, 0.01, 32)
    for r in (a, b):
        r.update(R=2, steps=100, measure_every=10, tau_walk=[3.0] * 40)
        r["means"] = {k: np.asarray(v) for k, v in r["means"].items()}
    fss.save_runs(tmp_path / "x.npz", [a, b])
    out = subprocess.run([sys.executable, "-m", "paper_1309_1599_amd.fss", "--combine", str(tmp_path / "x.npz"),
                          "--out", str(tmp_path / "x.json")], capture_output=True, text=True, timeout=120,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert out.returncode == 0, out.stderr
    line = json.loads(out.stdout)
    assert line["samples"] == [40, 40] and line["crossings"][0]["channel"] == "sg"
    rep = json.loads((tmp_path / "x.json").read_text())
    assert rep["crossings"][0]["T_cross"][0] == pytest.approx(0.95, abs=0.02)
    assert rep["temperature_walk"]["16"]["runs_longer_than_10_tau"] == 1.0


def test_simulate_host_logic_with_a_scripted_library(monkeypatch):
    """fss.simulate's bookkeeping on the CPU: the library calls are replaced
    by a scripted stand-in whose records carry known overlaps, so the bin
    means, counts and walk times can be checked exactly."""
    from paper_1309_1599_amd import ptsg
    L, S, R, steps, every = 4, 3, 2, 64, 2
    temps = np.linspace(1.0, 2.0, 5)
    T, N = len(temps), L ** 3
    state = {"m": 0}
    rng = np.random.default_rng(9)

    def q_of(s, k, m):
        return 0.1 * (s + 1) + 0.01 * k + 0.001 * m

    def init(Ls, cpl, ts, n_rep, seed, flags=0):
        assert Ls == [L] * S and n_rep == R and len(cpl) == S and flags & ptsg.PT_F_BIMODAL
        state["perm"] = np.stack([np.stack([np.arange(T)] * R)] * S)
        return "ctx"

    def swap(ctx):
        state["perm"] = np.stack([np.stack([rng.permutation(T) for _ in range(R)]) for _ in range(S)])

    def measure(ctx, what):
        assert what & ptsg.PT_M_OVERLAP and what & ptsg.PT_M_CHIRAL
        out = np.zeros(S * T, ptsg.MEAS_DTYPE)
        for i, (s, k) in enumerate((s, k) for s in range(S) for k in range(T)):
            out[i]["sample"], out[i]["tslot"], out[i]["rep_b"] = s, k, 1
            out[i]["q0"][0] = q_of(s, k, state["m"])
            out[i]["qk_re"][:, 0] = 0.2
            out[i]["cg0"] = 0.05 * (k + 1)
            out[i]["E_a"] = out[i]["E_b"] = -(k + 1.0) * N
        state["m"] += 1
        return out

    monkeypatch.setattr(ptsg, "pt_init_batch", init)
    monkeypatch.setattr(ptsg, "pt_step", lambda ctx, n_hb, n_or: None)
    monkeypatch.setattr(ptsg, "pt_swap", swap)
    monkeypatch.setattr(ptsg, "pt_measure", measure)
    monkeypatch.setattr(ptsg, "pt_get_perms", lambda ctx: list(state["perm"]))
    monkeypatch.setattr(ptsg, "pt_free", lambda ctx: None)
    run = fss.simulate(L, S, temps, R, steps, every, 5, "bimodal", 1.0, chiral=True, log=lambda msg: None)
    n = steps // every
    assert run["bins"][0] == (n // 2, n) and run["counts"][0] == n // 2
    last = range(n // 2, n)
    for s in range(S):
        for k in range(T):
            want = np.mean([q_of(s, k, m) ** 2 for m in last])
            assert run["means"]["q2"][0][s][k] == pytest.approx(want, rel=1e-12)
            assert run["means"]["qk2"][0][s][k] == pytest.approx(0.04, rel=1e-12)
            assert run["means"]["cg2"][0][s][k] == pytest.approx((0.05 * (k + 1)) ** 2, rel=1e-12)
            assert run["means"]["e"][0][s][k] == pytest.approx(-(k + 1.0), rel=1e-12)
    # a fresh random permutation at every swap: the slots are uncorrelated in time
    assert len(run["tau_walk"]) == S
    assert all(0.3 < t / every < 0.8 for t in run["tau_walk"]), run["tau_walk"]


def _table1():
    import csv
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_run_parameters.csv")
    with open(path) as fh:
        rows = [r for r in csv.DictReader(line for line in fh if not line.startswith("#"))]
    return {(float(r["D"]), int(r["L"])): r for r in rows}


def test_cli_defaults_follow_table_1():
    """The driver's defaults are the paper's D = 1 protocol at L = 8 and 16
    (Table I): T in [0.877, 1.28], 20480 and 40960 MCS, two replicas, and the
    28 temperatures Table I gives for L = 16 (Table I gives 10 at L = 8; the
    driver puts both sizes on the larger grid, since the crossing fits compare
    the two sizes at the same temperatures)."""
    t1 = _table1()
    args = fss.make_parser().parse_args([])
    assert args.L == [8, 16] and args.replicas == 2 and args.D == 1.0 and args.couplings == "bimodal"
    for L, steps in zip(args.L, args.steps):
        row = t1[(1.0, L)]
        assert steps == int(row["n_mcs_min"])
        assert args.temps[0] == float(row["T_min"]) and args.temps[1] == float(row["T_max"])
    assert args.temps[2] == int(t1[(1.0, 16)]["n_temps"])
    # the D = 0.5 runs of the same sizes use Table I's grid and lengths through the options
    row8, row16 = t1[(0.5, 8)], t1[(0.5, 16)]
    assert (row8["T_min"], row8["T_max"]) == (row16["T_min"], row16["T_max"]) == ("0.588", "0.8")
    assert (int(row8["n_mcs_min"]), int(row16["n_mcs_min"])) == (20480, 40960)
