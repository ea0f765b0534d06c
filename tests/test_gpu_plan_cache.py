"""The autotuner's plan cache on disk (PTSG_PLAN_CACHE): a tuning result (the
mapping and its tile shape) is appended as one line, a matching line is used
instead of timing, and lines that do not parse or name a mapping the lattice
cannot use are skipped."""
import numpy as np
import pytest

from paper_1309_1599_amd import inputs, ptsg

pytestmark = pytest.mark.gpu

NAME = {ptsg.PT_F_SITE_LANES: "site", ptsg.PT_F_CHAIN_LANES: "chain", ptsg.PT_F_RESIDENT: "resident"}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    ptsg.load_library()


def _tuned(L, T, seed, flags=0):
    temps = inputs.geometric_temps(0.8, 1.6, T)
    if flags & ptsg.PT_F_BIMODAL:
        M = inputs.bimodal_couplings(L, 1.0, seed)
    else:
        M = inputs.gaussian_couplings(L, seed)
    ctx = ptsg.pt_init_batch([L], [M], [temps], 2, seed, flags=ptsg.PT_F_AUTOTUNE | flags)
    m = ptsg.pt_get_mapping(ctx, 0)
    tile = ptsg.pt_get_tile(ctx, 0)
    ptsg.pt_step(ctx, 1, 2)
    e = ptsg.pt_get_energy(ctx)
    ptsg.pt_free(ctx)
    assert np.isfinite(e).all()
    return m, tile


def test_plan_cache_file(tmp_path, monkeypatch):
    path = tmp_path / "plans.txt"
    monkeypatch.setenv("PTSG_PLAN_CACHE", str(path))
    # temperature counts no other test tunes, so the process cache is empty for them
    chosen, tile = _tuned(8, 5, 801)
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    f = lines[0].split()
    assert len(f) == 14 and f[0] == "ptsg-plan" and f[1] == "2"
    assert f[4:10] == ["8", "5", "2", "1", "0", "0"] and f[10] == NAME[chosen]
    if chosen == ptsg.PT_F_SITE_LANES:
        assert int(f[11]) == tile[0]
    if chosen == ptsg.PT_F_CHAIN_LANES:
        assert (int(f[12]), int(f[13])) == tile[1:]

    # a line for a key not yet tuned is used as it stands, tile shape included
    forged = f[:5] + ["7"] + f[6:10] + ["site", "3", "0", "-1"]
    path.write_text(lines[0] + "\nnot a plan line\n" + " ".join(f[:5] + ["7"] + f[6:10] + ["site", "3"]) + "\n"
                    + " ".join(forged) + "\n")
    assert _tuned(8, 7, 802) == (ptsg.PT_F_SITE_LANES, (3, 0, 0))
    assert len(path.read_text().splitlines()) == 4          # nothing appended

    # "resident" cannot hold L = 24: the line is skipped and the class is timed
    bad = f[:4] + ["24", "9"] + f[6:10] + ["resident", "0", "0", "-1"]
    path.write_text(" ".join(bad) + "\n")
    got, _ = _tuned(24, 9, 803)
    assert got in (ptsg.PT_F_SITE_LANES, ptsg.PT_F_CHAIN_LANES)
    lines = path.read_text().splitlines()
    assert len(lines) == 2 and lines[1].split()[10] == NAME[got]


def test_plan_cache_bimodal_key(tmp_path, monkeypatch):
    """Bimodal samples are tuned in their byte coding, under their own key."""
    path = tmp_path / "plans.txt"
    monkeypatch.setenv("PTSG_PLAN_CACHE", str(path))
    chosen, _ = _tuned(8, 11, 804, ptsg.PT_F_BIMODAL)
    f = path.read_text().split()
    assert f[4:10] == ["8", "11", "2", "1", "0", "1"] and f[10] == NAME[chosen]
