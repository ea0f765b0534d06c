"""CPU checks of the C ABI: the library loads, exports every entry point
include/ptsg.h declares, and rejects invalid arguments before touching a
device (no kernel is launched here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1309_1599_amd import inputs, ptsg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptsg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ptsg.LIB_PATH):
        from paper_1309_1599_amd import build
        build.build()
    return ptsg.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert "pt_init" in names and "pt_measure" in names
    assert sorted(ptsg.EXPORTS) == names
    for n in names:
        assert hasattr(lib, n), n


def test_meas_record_layout():
    assert ptsg.MEAS_DTYPE.itemsize == 744
    assert ptsg.MEAS_DTYPE.fields["beta"][1] == 16
    assert ptsg.MEAS_DTYPE.fields["sd2_b"][1] == 744 - 8


def test_workspace_size_accounts_for_state(lib):
    L, T, R = 16, 4, 2
    cpl = [inputs.gaussian_couplings(L, 1)]
    n = ptsg.pt_workspace_size([L], cpl, [inputs.geometric_temps(0.5, 1.5, T)], R)
    N = L ** 3
    spins = 4 * 3 * N * T * R
    couplings = 4 * 54 * N
    assert n >= spins + couplings
    assert n < 2 * (spins + couplings) + (1 << 20)


@pytest.mark.parametrize("L,temps,R,why", [
    (5, [1.0, 2.0], 2, "L must be even"),
    (2, [1.0, 2.0], 2, "L must be even"),
    (8, [2.0, 1.0], 2, "strictly ascending"),
    (8, [1.0, 1.0], 2, "strictly ascending"),
    (8, [-1.0, 1.0], 2, "> 0"),
    (8, [1.0, 2.0], 0, "n_replicas"),
    (8, [], 2, "n_temps"),
])
def test_invalid_arguments_rejected(lib, L, temps, R, why):
    cpl = np.zeros((3, L ** 3, 3, 3), np.float32)
    assert ptsg.pt_workspace_size([L], [cpl], [temps], R) == 0
    with pytest.raises(ptsg.PtError) as e:
        ptsg.pt_init(L, cpl, temps, R, 1)
    assert e.value.status == ptsg.PT_EINVAL
    assert why in str(e.value)


def test_non_finite_coupling_rejected(lib):
    L = 4
    cpl = np.zeros((3, L ** 3, 3, 3), np.float32)
    cpl[1, 7, 2, 0] = np.nan
    with pytest.raises(ptsg.PtError) as e:
        ptsg.pt_init(L, cpl, [1.0], 1, 1)
    assert e.value.status == ptsg.PT_EINVAL and "non-finite" in str(e.value)


def test_null_context_is_state_error(lib):
    assert lib.pt_step(None, 1, 1) == ptsg.PT_ESTATE
    assert lib.pt_swap(None) == ptsg.PT_ESTATE
    assert lib.pt_get_perms(None, None) == ptsg.PT_ESTATE
    assert "pt_init" in ptsg.pt_last_error()
    lib.pt_free(None)  # no-op


def test_workspace_reflects_mapping(lib):
    """Chain lanes pad a sample's chains to whole 64-lane groups and stage
    all chains of the sample in the site-lane layout for measurements (other
    mappings stage one chain); every mapping keeps 54 packed coupling floats
    per site (in its own order).  (Plan only: no device is touched.)"""
    L, T, R = 24, 35, 2          # 70 chains -> 2 groups of 64 lanes
    N = L ** 3
    cpl = [np.zeros((3, N, 3, 3), np.float32)]
    temps = [inputs.geometric_temps(0.5, 1.5, T)]
    site = ptsg.pt_workspace_size([L], cpl, temps, R, flags=ptsg.PT_F_SITE_LANES)
    chain = ptsg.pt_workspace_size([L], cpl, temps, R, flags=ptsg.PT_F_CHAIN_LANES)
    plain = ptsg.pt_workspace_size([L], cpl, temps, R, flags=ptsg.PT_F_PLAIN)
    assert site == plain
    spins_site, spins_chain = 4 * 3 * N * 70, 4 * 3 * N * 128
    stage_extra = 4 * 3 * N * (70 - 1)
    assert chain - site == pytest.approx(spins_chain - spins_site + stage_extra, abs=1 << 20)
    # resident needs L <= 16; otherwise the sample falls back to site lanes
    assert ptsg.pt_workspace_size([L], cpl, temps, R, flags=ptsg.PT_F_RESIDENT) == site
    small = [np.zeros((3, 512, 3, 3), np.float32)]
    assert (ptsg.pt_workspace_size([8], small, temps, R, flags=ptsg.PT_F_RESIDENT)
            == ptsg.pt_workspace_size([8], small, temps, R, flags=ptsg.PT_F_SITE_LANES))


def test_autotune_ignored_when_mapping_forced(lib):
    """A mapping flag or the plain form switches the autotuner off, so the
    plan (and its size) is the forced one and no device is needed."""
    L, T, R = 24, 35, 2
    cpl = [np.zeros((3, L ** 3, 3, 3), np.float32)]
    temps = [inputs.geometric_temps(0.5, 1.5, T)]
    for f in (ptsg.PT_F_SITE_LANES, ptsg.PT_F_CHAIN_LANES, ptsg.PT_F_PLAIN):
        assert (ptsg.pt_workspace_size([L], cpl, temps, R, flags=f | ptsg.PT_F_AUTOTUNE)
                == ptsg.pt_workspace_size([L], cpl, temps, R, flags=f))


def test_checkpoint_calls_need_a_context(lib):
    n = C.c_size_t()
    assert lib.pt_save(None, None, 0, C.byref(n)) == ptsg.PT_ESTATE
    assert lib.pt_load(None, None, 0) == ptsg.PT_ESTATE


def test_bimodal_flag_validates_the_family(lib):
    """PT_F_BIMODAL accepts the paper's family bit for bit (D = 0.5 and D = 1,
    where diagonals can be exactly 0) and stores 8 bytes of codes per site
    for site-lane and chain-lane samples instead of 54 floats (plus the
    sample's table of 128 code matrices); anything else is refused."""
    L, T, R = 8, 4, 2
    N = L ** 3
    temps = [inputs.geometric_temps(0.5, 1.5, T)]
    for f in (ptsg.PT_F_SITE_LANES, ptsg.PT_F_CHAIN_LANES):
        for D in (0.5, 1.0):
            cpl = [inputs.bimodal_couplings(L, D, 3)]
            plain = ptsg.pt_workspace_size([L], cpl, temps, R, flags=f)
            packed = ptsg.pt_workspace_size([L], cpl, temps, R, flags=f | ptsg.PT_F_BIMODAL)
            assert packed > 0
            assert plain - packed == pytest.approx(4 * (54 - 2) * N - 4 * 128 * 9, abs=1024)
    # the resident kernel keeps the floats: only the table is added
    cpl = [inputs.bimodal_couplings(L, 0.5, 3)]
    plain = ptsg.pt_workspace_size([L], cpl, temps, R, flags=ptsg.PT_F_RESIDENT)
    packed = ptsg.pt_workspace_size([L], cpl, temps, R, flags=ptsg.PT_F_RESIDENT | ptsg.PT_F_BIMODAL)
    assert packed - plain == pytest.approx(4 * 128 * 9, abs=512)

    def refused(M):
        ok = ptsg.pt_workspace_size([L], [M], temps, R, flags=ptsg.PT_F_BIMODAL) > 0
        return not ok and "PT_F_BIMODAL" in ptsg.pt_last_error()

    assert refused(inputs.gaussian_couplings(L, 3))
    base = inputs.bimodal_couplings(L, 1.0, 4)
    M = base.copy()
    M[1, 17, 0, 1] = -M[1, 17, 0, 1]          # asymmetric bond
    assert refused(M)
    M = base.copy()
    M[2, 5, 1, 2] = M[2, 5, 2, 1] = 0.25      # another magnitude
    assert refused(M)
    M = base.copy()
    mu, i, a = np.argwhere(M[..., [0, 1, 2], [0, 1, 2]] == 0)[0]   # D = 1: exact zeros
    M[mu, i, a, a] = -0.0                     # equal as a number, other bits
    assert refused(M)


def test_row_order_flag_validation(lib):
    temps = [inputs.geometric_temps(0.5, 1.5, 3)]
    ok = ptsg.pt_workspace_size([16], [np.zeros((3, 16 ** 3, 3, 3), np.float32)], temps, 2,
                                flags=ptsg.PT_F_ROW_OR)
    assert ok > 0
    for L, flags in ((12, ptsg.PT_F_ROW_OR), (24, ptsg.PT_F_ROW_OR), (40, ptsg.PT_F_ROW_OR),
                     (16, ptsg.PT_F_ROW_OR | ptsg.PT_F_SITE_LANES),
                     (16, ptsg.PT_F_ROW_OR | ptsg.PT_F_PLAIN)):
        cpl = [np.zeros((3, L ** 3, 3, 3), np.float32)]
        assert ptsg.pt_workspace_size([L], cpl, temps, 2, flags=flags) == 0
        assert "PT_F_ROW_OR" in ptsg.pt_last_error()
