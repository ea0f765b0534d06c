"""ctypes binding of the FP64 oracle library (liboracle.so).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each function is a
thin call into the C routine of the same name; arrays are float64 in the
canonical layouts: couplings [3][N][3][3], spins [N][3].
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

_dp = C.POINTER(C.c_double)
_u32p = C.POINTER(C.c_uint32)
_i32p = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.or_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.or_neighbour.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_neighbour.restype = C.c_int
        L.or_local_field.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp]
        L.or_energy.argtypes = [C.c_int, _dp, _dp]
        L.or_energy.restype = C.c_double
        L.or_heatbath_spin.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp]
        L.or_overrelax_spin.argtypes = [_dp, _dp]
        L.or_u23.argtypes = [C.c_uint32]
        L.or_u23.restype = C.c_double
        L.or_u52.argtypes = [C.c_uint32, C.c_uint32]
        L.or_u52.restype = C.c_double
        L.or_ctr3.argtypes = [C.c_uint32] * 3
        L.or_ctr3.restype = C.c_uint32
        L.or_half_sweep.argtypes = [C.c_int, _dp, _dp, C.c_int, C.c_int, C.c_double,
                                    C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                    C.c_uint32]
        L.or_init_spins.argtypes = [C.c_int, _dp, C.c_uint64, C.c_uint32, C.c_uint32,
                                    C.c_uint32]
        L.or_row_sweep.argtypes = [C.c_int, _dp, _dp]
        L.or_row_sweep.restype = C.c_int
        L.or_pt_pass.argtypes = [C.c_int, _dp, _dp, _i32p, C.c_uint64, C.c_uint32,
                                 C.c_uint32, C.c_uint32]
        L.or_pt_pass.restype = C.c_int
        L.or_overlaps.argtypes = [C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_sd_sums.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


TAG_HB, TAG_PT, TAG_INIT = 0, 1, 2


def philox(key, ctr):
    k = np.ascontiguousarray(key, dtype=np.uint32)
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(k.ctypes.data_as(_u32p), c.ctypes.data_as(_u32p),
                           out.ctypes.data_as(_u32p))
    return out


def neighbour(L, i, mu, direction):
    return lib().or_neighbour(L, i, mu, direction)


def local_field(L, M, s, i):
    M, s = _f64(M), _f64(s)
    h = np.zeros(3)
    lib().or_local_field(L, _d(M), _d(s), i, _d(h))
    return h


def local_fields(L, M, s):
    """h for every site, [N][3] (loop over or_local_field)."""
    N = L ** 3
    return np.stack([local_field(L, M, s, i) for i in range(N)])


def energy(L, M, s):
    M, s = _f64(M), _f64(s)
    return lib().or_energy(L, _d(M), _d(s))


def heatbath_spin(h, beta, v, u2):
    h = _f64(h)
    s = np.zeros(3)
    lib().or_heatbath_spin(_d(h), float(beta), float(v), float(u2), _d(s))
    return s


def overrelax_spin(h, s):
    h, s = _f64(h), _f64(s).copy()
    lib().or_overrelax_spin(_d(h), _d(s))
    return s


def u23(w):
    return lib().or_u23(int(w))


def u52(w0, w1):
    return lib().or_u52(int(w0), int(w1))


def ctr3(tag, tslot, rep):
    return lib().or_ctr3(tag, tslot, rep)


def half_sweep(L, M, s, colour, kind, beta, seed, hb_sweep, sample, tslot, rep):
    """In place on s (float64 [N][3], C-contiguous)."""
    assert s.dtype == np.float64 and s.flags.c_contiguous
    M = _f64(M)
    lib().or_half_sweep(L, _d(M), _d(s), colour, kind, float(beta), int(seed),
                        int(hb_sweep), int(sample), int(tslot), int(rep))


def sweep(L, M, s, kind, beta, seed, hb_sweep, sample, tslot, rep):
    """Colour 0 then colour 1."""
    for c in (0, 1):
        half_sweep(L, M, s, c, kind, beta, seed, hb_sweep, sample, tslot, rep)


def init_spins(L, seed, sample, chain, rep):
    s = np.zeros((L ** 3, 3))
    lib().or_init_spins(L, _d(s), int(seed), int(sample), int(chain), int(rep))
    return s


def pt_pass(beta, E, perm, seed, pass_index, sample, rep):
    """One PT pass; perm (int32 [T], slot -> chain) is updated in place.
    Returns the number of accepted swaps."""
    beta, E = _f64(beta), _f64(E)
    assert perm.dtype == np.int32 and perm.flags.c_contiguous
    return lib().or_pt_pass(len(beta), _d(beta), _d(E), perm.ctypes.data_as(_i32p),
                            int(seed), int(pass_index), int(sample), int(rep))


def row_sweep(L, M, s):
    """Row-ordered overrelaxation sweep, in place (s: float64 [N][3]).
    L must be 8 or a multiple of 16 (ValueError otherwise: for an odd number
    of 8-site rows along x above one, two rows of one class touch)."""
    assert s.dtype == np.float64 and s.flags.c_contiguous
    M = _f64(M)
    if lib().or_row_sweep(L, _d(M), _d(s)) != 0:
        raise ValueError(f"row order needs L = 8 or a multiple of 16, got L = {L}")


def overlaps(L, sa, sb):
    sa, sb = _f64(sa), _f64(sb)
    q0 = np.zeros(9); qr = np.zeros(27); qi = np.zeros(27)
    c0 = np.zeros(3); cr = np.zeros(9); ci = np.zeros(9)
    lib().or_overlaps(L, _d(sa), _d(sb), _d(q0), _d(qr), _d(qi), _d(c0), _d(cr), _d(ci))
    return dict(q0=q0, qk_re=qr.reshape(3, 9), qk_im=qi.reshape(3, 9), cg0=c0,
                cgk_re=cr.reshape(3, 3), cgk_im=ci.reshape(3, 3))


def sd_sums(L, M, s):
    M, s = _f64(M), _f64(s)
    a = C.c_double(); b = C.c_double()
    lib().or_sd_sums(L, _d(M), _d(s), C.byref(a), C.byref(b))
    return a.value, b.value
