"""Python binding of libptsg.so (include/ptsg.h), argument marshalling only.

Every function has the name and meaning of the C entry point it wraps.
PyTorch supplies the device memory (the workspace tensor) and the stream;
all computation runs in the library's HIP kernels.  There is no fallback:
without the built library or a GPU these functions raise.
"""
import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libptsg.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_ESTATE, PT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PT_M_OVERLAP, PT_M_CHIRAL, PT_M_SD, PT_M_ENERGY, PT_M_ALL = 1, 2, 4, 8, 15
PT_K_OVERRELAX, PT_K_HEATBATH, PT_K_RESIDENT, PT_K_PERSISTENT = 0, 1, 2, 3
PT_F_SITE_LANES, PT_F_CHAIN_LANES, PT_F_RESIDENT, PT_F_GRAPHS, PT_F_PLAIN, PT_F_AUTOTUNE, PT_F_BIMODAL = \
    1, 2, 4, 8, 16, 32, 64
PT_F_ROW_OR = 128
PT_F_PERSISTENT = 256
PT_OR_L = -1   # pt_step: L overrelaxation sweeps for a sample of linear size L

# numpy view of the C struct pt_meas (744 bytes, no padding)
MEAS_DTYPE = np.dtype([
    ("sample", "<i4"), ("tslot", "<i4"), ("rep_a", "<i4"), ("rep_b", "<i4"),
    ("beta", "<f8"), ("E_a", "<f8"), ("E_b", "<f8"),
    ("q0", "<f8", (9,)), ("qk_re", "<f8", (3, 9)), ("qk_im", "<f8", (3, 9)),
    ("cg0", "<f8", (3,)), ("cgk_re", "<f8", (3, 3)), ("cgk_im", "<f8", (3, 3)),
    ("sd1_a", "<f8"), ("sd2_a", "<f8"), ("sd1_b", "<f8"), ("sd2_b", "<f8"),
])
assert MEAS_DTYPE.itemsize == 744

# Every symbol the C ABI exports (include/ptsg.h).
EXPORTS = ["pt_init", "pt_workspace_size", "pt_init_batch", "pt_step", "pt_swap", "pt_measure",
           "pt_measure_noalloc", "pt_run",
           "pt_get_spins", "pt_set_spins", "pt_get_perm", "pt_get_perms", "pt_get_energy", "pt_get_counters",
           "pt_set_stream", "pt_sync", "pt_profile", "pt_kernel_time", "pt_get_mapping", "pt_get_tile",
           "pt_save", "pt_load", "pt_free", "pt_last_error"]


class PtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ptsg error {status}: {msg}")
        self.status = status


class pt_batch_desc(C.Structure):
    _fields_ = [("n_samples", C.c_int),
                ("L", C.POINTER(C.c_int)),
                ("n_temps", C.POINTER(C.c_int)),
                ("temps", C.POINTER(C.POINTER(C.c_double))),
                ("couplings", C.POINTER(C.POINTER(C.c_float))),
                ("n_replicas", C.c_int),
                ("seed", C.c_uint64),
                ("stream", C.c_void_p),
                ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t),
                ("flags", C.c_uint)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libptsg.so (torch is imported first so that one HIP runtime is shared)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1309_1599_amd.build`")
    import torch  # noqa: F401  (HIP runtime of torch becomes the process's runtime)
    lib = C.CDLL(path)
    vp, i, u64, sz = C.c_void_p, C.c_int, C.c_uint64, C.c_size_t
    sig = {
        "pt_init": (i, [C.POINTER(vp), i, C.POINTER(C.c_float), C.POINTER(C.c_double), i, i, u64]),
        "pt_workspace_size": (sz, [C.POINTER(pt_batch_desc)]),
        "pt_init_batch": (i, [C.POINTER(vp), C.POINTER(pt_batch_desc)]),
        "pt_step": (i, [vp, i, i]),
        "pt_swap": (i, [vp]),
        "pt_measure": (i, [vp, C.c_uint, vp, sz, C.POINTER(sz)]),
        "pt_measure_noalloc": (i, [vp, C.c_uint, vp, sz]),
        "pt_run": (i, [vp, i, i, i, i, C.c_uint, vp, sz]),
        "pt_get_spins": (i, [vp, i, i, i, C.POINTER(C.c_float)]),
        "pt_set_spins": (i, [vp, i, i, i, C.POINTER(C.c_float)]),
        "pt_get_perm": (i, [vp, i, i, C.POINTER(C.c_int32)]),
        "pt_get_perms": (i, [vp, C.POINTER(C.c_int32)]),
        "pt_get_energy": (i, [vp, C.POINTER(C.c_double)]),
        "pt_get_counters": (i, [vp, C.POINTER(u64), C.POINTER(u64)]),
        "pt_set_stream": (i, [vp, vp]),
        "pt_sync": (i, [vp]),
        "pt_profile": (i, [vp, i]),
        "pt_kernel_time": (i, [vp, i, C.POINTER(u64), C.POINTER(C.c_double)]),
        "pt_get_mapping": (i, [vp, i, C.POINTER(C.c_uint)]),
        "pt_get_tile": (i, [vp, i, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "pt_save": (i, [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]),
        "pt_load": (i, [vp, vp, C.c_size_t]),
        "pt_free": (None, [vp]),
        "pt_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def pt_last_error():
    return load_library().pt_last_error().decode()


def _check(status):
    if status != PT_OK:
        raise PtError(status, pt_last_error())


class PtContext:
    """Handle of a pt_ctx plus the host-side facts the binding needs."""

    def __init__(self, ptr, L, n_temps, n_replicas, workspace=None):
        self.ptr = C.c_void_p(ptr)
        self.L = list(L)
        self.n_temps = list(n_temps)
        self.n_replicas = n_replicas
        self.workspace = workspace  # torch tensor kept alive with the context

    @property
    def n_samples(self):
        return len(self.L)

    @property
    def n_records(self):
        R = self.n_replicas
        return sum(T * R * (R - 1) // 2 for T in self.n_temps)

    @property
    def n_chains(self):
        return sum(T * self.n_replicas for T in self.n_temps)

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: the
        # process is ending and the driver releases the device memory
        if getattr(self, "ptr", None) is not None and self.ptr.value and pt_free is not None:
            try:
                pt_free(self)
            except Exception:
                pass


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _desc(L, couplings, temps, n_replicas, seed, stream=None, workspace=None, nbytes=0, flags=0):
    S = len(L)
    keep = [_f32(c).reshape(-1) for c in couplings], [_f64(t) for t in temps]
    Ls = (C.c_int * S)(*[int(x) for x in L])
    Ts = (C.c_int * S)(*[len(t) for t in keep[1]])
    tp = (C.POINTER(C.c_double) * S)(*[t.ctypes.data_as(C.POINTER(C.c_double)) for t in keep[1]])
    cp = (C.POINTER(C.c_float) * S)(*[c.ctypes.data_as(C.POINTER(C.c_float)) for c in keep[0]])
    d = pt_batch_desc(S, Ls, Ts, tp, cp, int(n_replicas), int(seed) & (2 ** 64 - 1),
                      stream, workspace, nbytes, int(flags))
    return d, (keep, Ls, Ts, tp, cp)


def pt_workspace_size(L, couplings, temps, n_replicas, seed=0, flags=0):
    d, _keep = _desc(L, couplings, temps, n_replicas, seed, flags=flags)
    return load_library().pt_workspace_size(C.byref(d))


def pt_init_batch(L, couplings, temps, n_replicas, seed, stream=None, device=None, flags=0):
    """Batch of samples: L[s], couplings[s] ([3][L^3][3][3] float32), temps[s].
    The workspace is a torch uint8 tensor on `device` (default: current);
    work goes to `stream` (default: torch's current stream); `flags` are the
    PT_F_* mapping choices (0 = automatic)."""
    import torch
    lib = load_library()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    with torch.cuda.device(dev):
        nbytes = pt_workspace_size(L, couplings, temps, n_replicas, seed, flags)
        if nbytes == 0:
            d, _k = _desc(L, couplings, temps, n_replicas, seed, flags=flags)
            h = C.c_void_p()
            _check(lib.pt_init_batch(C.byref(h), C.byref(d)))  # raises with the reason
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        st = (stream if stream is not None else torch.cuda.current_stream(dev)).cuda_stream
        d, _keep = _desc(L, couplings, temps, n_replicas, seed, C.c_void_p(st),
                         C.c_void_p(ws.data_ptr()), nbytes, flags)
        h = C.c_void_p()
        _check(lib.pt_init_batch(C.byref(h), C.byref(d)))
    return PtContext(h.value, L, [len(t) for t in temps], n_replicas, ws)


def pt_init(L, couplings, temps, n_replicas, seed):
    """Single sample; library-owned memory, null stream."""
    lib = load_library()
    cpl = _f32(couplings).reshape(-1)
    t = _f64(temps)
    h = C.c_void_p()
    _check(lib.pt_init(C.byref(h), int(L), cpl.ctypes.data_as(C.POINTER(C.c_float)),
                       t.ctypes.data_as(C.POINTER(C.c_double)), len(t), int(n_replicas),
                       int(seed) & (2 ** 64 - 1)))
    return PtContext(h.value, [L], [len(t)], n_replicas)


def pt_step(ctx, n_hb, n_or):
    _check(load_library().pt_step(ctx.ptr, int(n_hb), int(n_or)))


def pt_swap(ctx):
    _check(load_library().pt_swap(ctx.ptr))


def pt_measure(ctx, what=PT_M_ALL):
    out = np.zeros(max(1, ctx.n_records), dtype=MEAS_DTYPE)
    n = C.c_size_t()
    _check(load_library().pt_measure(ctx.ptr, int(what), out.ctypes.data_as(C.c_void_p),
                                     len(out), C.byref(n)))
    return out[: n.value]


def pt_run(ctx, n_steps, n_hb, n_or, every=0, what=PT_M_ALL, d_out=0, cap=0):
    """n_steps whole steps (sweeps + tempering, a measurement every `every`
    steps into the device array at address d_out with room for cap records);
    asynchronous."""
    _check(load_library().pt_run(ctx.ptr, int(n_steps), int(n_hb), int(n_or), int(every), int(what),
                                 C.c_void_p(int(d_out)) if d_out else None, int(cap)))


def pt_measure_noalloc(ctx, what, d_out, cap):
    """Records into a device buffer (address d_out, room for cap records),
    queued on the context's stream; nothing is allocated or copied."""
    _check(load_library().pt_measure_noalloc(ctx.ptr, int(what), C.c_void_p(int(d_out)), int(cap)))


def pt_get_spins(ctx, sample, rep, tslot):
    N = ctx.L[sample] ** 3
    out = np.empty((N, 3), dtype=np.float32)
    _check(load_library().pt_get_spins(ctx.ptr, sample, rep, tslot,
                                       out.ctypes.data_as(C.POINTER(C.c_float))))
    return out


def pt_set_spins(ctx, sample, rep, tslot, spins):
    s = _f32(spins).reshape(-1)
    assert s.size == 3 * ctx.L[sample] ** 3
    _check(load_library().pt_set_spins(ctx.ptr, sample, rep, tslot,
                                       s.ctypes.data_as(C.POINTER(C.c_float))))


def pt_get_perm(ctx, sample, rep):
    out = np.empty(ctx.n_temps[sample], dtype=np.int32)
    _check(load_library().pt_get_perm(ctx.ptr, sample, rep,
                                      out.ctypes.data_as(C.POINTER(C.c_int32))))
    return out


def pt_get_perms(ctx):
    """Permutations of every (sample, replica): list of [R][T] int32 arrays,
    entry [r][k] = chain at slot k."""
    out = np.empty(ctx.n_chains, dtype=np.int32)
    _check(load_library().pt_get_perms(ctx.ptr, out.ctypes.data_as(C.POINTER(C.c_int32))))
    res, o = [], 0
    for T in ctx.n_temps:
        res.append(out[o:o + ctx.n_replicas * T].reshape(ctx.n_replicas, T))
        o += ctx.n_replicas * T
    return res


def pt_get_energy(ctx):
    """Energies ordered by (sample, replica, slot); list of [R][T] arrays."""
    out = np.empty(ctx.n_chains, dtype=np.float64)
    _check(load_library().pt_get_energy(ctx.ptr, out.ctypes.data_as(C.POINTER(C.c_double))))
    res, o = [], 0
    for T in ctx.n_temps:
        res.append(out[o:o + ctx.n_replicas * T].reshape(ctx.n_replicas, T))
        o += ctx.n_replicas * T
    return res


def pt_get_counters(ctx):
    a, b = C.c_uint64(), C.c_uint64()
    _check(load_library().pt_get_counters(ctx.ptr, C.byref(a), C.byref(b)))
    return a.value, b.value


def pt_set_stream(ctx, stream):
    _check(load_library().pt_set_stream(ctx.ptr, C.c_void_p(stream.cuda_stream if stream is not None
                                                             else 0)))


def pt_sync(ctx):
    _check(load_library().pt_sync(ctx.ptr))


def pt_profile(ctx, enable):
    _check(load_library().pt_profile(ctx.ptr, 1 if enable else 0))


def pt_kernel_time(ctx, kind):
    n, ms = C.c_uint64(), C.c_double()
    _check(load_library().pt_kernel_time(ctx.ptr, int(kind), C.byref(n), C.byref(ms)))
    return n.value, ms.value


def pt_get_mapping(ctx, sample):
    """PT_F_SITE_LANES, PT_F_CHAIN_LANES or PT_F_RESIDENT for `sample`."""
    f = C.c_uint()
    _check(load_library().pt_get_mapping(ctx.ptr, int(sample), C.byref(f)))
    return f.value


def pt_get_tile(ctx, sample):
    """(chains per workgroup, waves per packed row, y-rows per strip) of a sample's sweeps."""
    g, sp, sr = C.c_int(), C.c_int(), C.c_int()
    _check(load_library().pt_get_tile(ctx.ptr, int(sample), C.byref(g), C.byref(sp), C.byref(sr)))
    return g.value, sp.value, sr.value


def pt_save(ctx):
    """The context's whole Monte Carlo state as a numpy uint8 array."""
    lib = load_library()
    n = C.c_size_t()
    _check(lib.pt_save(ctx.ptr, None, 0, C.byref(n)))
    blob = np.empty(n.value, np.uint8)
    _check(lib.pt_save(ctx.ptr, blob.ctypes.data_as(C.c_void_p), blob.nbytes, C.byref(n)))
    return blob


def pt_load(ctx, blob):
    """Restore a state saved by pt_save into a context made from the same
    descriptor."""
    blob = np.ascontiguousarray(np.frombuffer(blob, np.uint8) if isinstance(blob, (bytes, bytearray))
                                else np.asarray(blob, np.uint8))
    _check(load_library().pt_load(ctx.ptr, blob.ctypes.data_as(C.c_void_p), blob.nbytes))


def pt_free(ctx):
    if ctx.ptr is not None and ctx.ptr.value:
        load_library().pt_free(ctx.ptr)
        ctx.ptr = C.c_void_p(None)
