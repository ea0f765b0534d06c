"""Host-side analysis of measurement records (Sec. II.B, Sec. III, Sec. IV).

Everything here is plain numpy on the records that `pt_measure` returns
(`ptsg.MEAS_DTYPE`), stacked over measurements into an array of shape
(n_meas, n_records):

* per-record fields: the scalar spin-glass overlap q = tr Q (the paper's
  q_x = s^a . s^b summed with e^{ik.x}/N, Sec. II.B), its modulus squared
  at the three smallest wave vectors, the chiral-glass overlaps q_CG^mu
  (averaged over mu and over the wave-vector directions, as the paper does),
  and the energy per spin;
* thermal averages per (sample, temperature slot) over measurements and
  replica pairs; disorder averages over samples;
* the second-moment correlation length of Sec. II.B,
  xi = sqrt(chi(0)/chi(k_min) - 1) / (2 sin(k_min/2)), k_min = 2 pi / L;
* the logarithmic binning of Sec. III (the last bin is the last half of the
  run, the one before it the second quarter, and so on) and the
  thermalisation test built on it;
* jackknife errors (Sec. IV) and the integrated autocorrelation time of a
  series, or of the temperature random walk of a sample's chains (Sec. III);
* the crossing temperature of xi_L/L and xi_2L/(2L) from low-order fits to
  the temperatures nearest to it, the exponent nu from the ratio of the
  slopes there and eta from the ratio of the susceptibilities there
  (Sec. IV, quotient method).
"""
import numpy as np

from .ptsg import MEAS_DTYPE


def records_from_dicts(recs):
    """Records given as dicts (field name -> value) as a MEAS_DTYPE array."""
    out = np.zeros(len(recs), MEAS_DTYPE)
    for i, r in enumerate(recs):
        for name in MEAS_DTYPE.names:
            if name in r:
                out[i][name] = r[name]
    return out


def stack(records_by_measurement):
    """(n_meas, n_records) array from a list of per-measurement record arrays
    (or lists of dicts)."""
    rows = [r if isinstance(r, np.ndarray) else records_from_dicts(r) for r in records_by_measurement]
    return np.stack(rows)


def _trace9(a):
    return a[..., 0] + a[..., 4] + a[..., 8]


def fields(R, L):
    """Per-measurement, per-record observables.  R: (n_meas, n_records)
    MEAS_DTYPE array; L: lattice size of every record (scalar, or an array
    over records).  Returns a dict of (n_meas, n_records) arrays:
    q (real q(0)), q2, q4, qk2 (|q(k_min)|^2 averaged over the 3 directions),
    cg2 (q_CG(0)^2 averaged over mu), cgk2 (|q_CG^mu(k_min)|^2 averaged over
    mu and directions) and e (energy per spin of the two replicas)."""
    N = np.asarray(L, dtype=np.float64) ** 3
    q = _trace9(R["q0"])
    qk2 = (_trace9(R["qk_re"]) ** 2 + _trace9(R["qk_im"]) ** 2).mean(axis=-1)
    cg2 = (R["cg0"] ** 2).mean(axis=-1)
    cgk2 = (R["cgk_re"] ** 2 + R["cgk_im"] ** 2).mean(axis=(-2, -1))
    e = (R["E_a"] + R["E_b"]) / (2.0 * N)
    return {"q": q, "q2": q ** 2, "q4": q ** 4, "qk2": qk2, "cg2": cg2, "cgk2": cgk2, "e": e}


def thermal_means(R, L, first=0, last=None):
    """Averages over measurements [first, last) and over the replica pairs of
    each (sample, slot).  Returns (keys, means) where keys is the list of
    (sample, slot) pairs and means maps each observable of `fields` to an
    array over keys."""
    F = fields(R[first:last], L)
    s, k = R["sample"][0], R["tslot"][0]
    keys = sorted(set(zip(s.tolist(), k.tolist())))
    index = {key: i for i, key in enumerate(keys)}
    which = np.array([index[(a, b)] for a, b in zip(s.tolist(), k.tolist())])
    counts = np.bincount(which, minlength=len(keys)).astype(np.float64)
    means = {}
    for name, v in F.items():
        per_rec = v.mean(axis=0)
        means[name] = np.bincount(which, weights=per_rec, minlength=len(keys)) / counts
    return keys, means


def xi_second_moment(chi0, chik, L):
    """Second-moment correlation length (Sec. II.B); 0 where chi(0) <= chi(k_min)."""
    ratio = np.maximum(np.asarray(chi0, dtype=np.float64) / np.asarray(chik, dtype=np.float64) - 1.0, 0.0)
    return np.sqrt(ratio) / (2.0 * np.sin(np.pi / np.asarray(L, dtype=np.float64)))


def susceptibilities(means, L):
    """chi_SG(0), chi_SG(k_min), chi_CG(0), chi_CG(k_min) = N <|q(k)|^2>
    from thermal (or disorder-averaged) means of `fields`."""
    N = np.asarray(L, dtype=np.float64) ** 3
    return {"chi_sg0": N * means["q2"], "chi_sgk": N * means["qk2"],
            "chi_cg0": N * means["cg2"], "chi_cgk": N * means["cgk2"]}


def jackknife(blocks, f=None):
    """Jackknife estimate and error of f(mean of blocks) over the first axis.
    blocks: (nb, ...) array of block means (nb >= 2); f defaults to the
    identity (then the error equals the standard error of the mean)."""
    blocks = np.asarray(blocks, dtype=np.float64)
    nb = blocks.shape[0]
    if nb < 2:
        raise ValueError("jackknife needs at least two blocks")
    f = f or (lambda m: m)
    total = blocks.sum(axis=0)
    full = f(total / nb)
    jk = np.stack([f((total - blocks[i]) / (nb - 1)) for i in range(nb)])
    err = np.sqrt((nb - 1) / nb * ((jk - jk.mean(axis=0)) ** 2).sum(axis=0))
    return full, err


def log_bins(n):
    """The logarithmic bins of a run of n measurements, last bin first:
    [n/2, n), [n/4, n/2), [n/8, n/4), ... down to a bin of one measurement
    (the first measurement of all, index 0, belongs to no bin)."""
    bins = []
    hi = n
    while hi >= 2:
        lo = hi // 2
        bins.append((lo, hi))
        hi = lo
    return bins


def thermalisation(series):
    """Sec. III test.  series: (n_meas, n_samples) per-sample values of one
    observable.  For every logarithmic bin i (last bin first), the disorder
    average of <O(i)> - <O(i_f)> and its jackknife error over samples.
    A run is thermalised when the differences of the last bins are
    compatible with zero."""
    series = np.asarray(series, dtype=np.float64)
    out = []
    bins = log_bins(series.shape[0])
    last = series[bins[0][0]:bins[0][1]].mean(axis=0)
    for lo, hi in bins:
        d = series[lo:hi].mean(axis=0) - last
        if d.shape[0] >= 2:
            m, e = jackknife(d[:, None])
            out.append((lo, hi, float(m[0]), float(e[0])))
        else:
            out.append((lo, hi, float(d.mean()), float("nan")))
    return out


def tau_int(x, c=6.0):
    """Integrated autocorrelation time tau = 1/2 + sum_{t>=1} rho(t) with
    Sokal's automatic window (the smallest W with W >= c tau(W)).  x is one
    series (n,) or several series of the same process (n, m), e.g. the
    temperature indices of all chains of a sample; their autocovariances
    (each about its own mean) are averaged before normalising."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    x = x - x.mean(axis=0)
    n = x.shape[0]
    if n < 2 or not np.any(x):
        return 0.5
    f = np.fft.rfft(x, 2 * n, axis=0)
    acf = np.fft.irfft(f * np.conj(f), 2 * n, axis=0)[:n].mean(axis=1)
    rho = acf / acf[0]
    tau = 0.5
    for w in range(1, n):
        tau += rho[w]
        if w >= c * tau:
            break
    return float(tau)


def slot_of_chain(perm):
    """Inverse of a permutation array (..., T): entry j = slot of chain j."""
    perm = np.asarray(perm)
    inv = np.empty_like(perm)
    np.put_along_axis(inv, perm, np.broadcast_to(np.arange(perm.shape[-1]), perm.shape), axis=-1)
    return inv


def temperature_walk_tau(slots):
    """Sec. III: integrated autocorrelation time of the random walk in
    temperature of one sample, in units of the sampling interval.
    slots: (n_times, n_chains) temperature index of every chain of the
    sample over time (all replicas)."""
    return tau_int(np.asarray(slots, dtype=np.float64))


def crossing(T, y1, y2, n_fit=4, order=1, extrapolate=0.0):
    """Temperature where curves y1(T) and y2(T) cross, from polynomial fits
    of degree `order` to the n_fit temperatures nearest to the crossing
    (Sec. IV: four temperatures, linear fits).  Returns (T_cross, y_cross,
    slope1, slope2).  If the curves do not cross inside the grid, the fits
    to the n_fit temperatures at the end where they come closest may place
    the crossing up to `extrapolate` times the width of the grid beyond it;
    otherwise (or farther out) ValueError."""
    T = np.asarray(T, dtype=np.float64)
    d = np.asarray(y1, dtype=np.float64) - np.asarray(y2, dtype=np.float64)
    sign = np.nonzero(np.diff(np.sign(d)) != 0)[0]
    width = T.max() - T.min()
    if len(sign) == 0:
        if extrapolate <= 0.0:
            raise ValueError("the curves do not cross in the temperature range")
        end = 0 if abs(d[0]) < abs(d[-1]) else len(T) - 1
        near = np.sort(np.argsort(np.abs(T - T[end]))[:n_fit])
        p1 = np.polyfit(T[near], np.asarray(y1)[near], 1)
        p2 = np.polyfit(T[near], np.asarray(y2)[near], 1)
        if p1[0] == p2[0]:
            raise ValueError("the curves do not cross in the temperature range")
        t0 = (p2[1] - p1[1]) / (p1[0] - p2[0])
        if not (T.min() - extrapolate * width <= t0 <= T.max() + extrapolate * width):
            raise ValueError("the curves do not cross near the temperature range")
    else:
        i = sign[0]
        t0 = T[i] - d[i] * (T[i + 1] - T[i]) / (d[i + 1] - d[i])
    near = np.sort(np.argsort(np.abs(T - t0))[:n_fit])
    p1 = np.polyfit(T[near], np.asarray(y1)[near], order)
    p2 = np.polyfit(T[near], np.asarray(y2)[near], order)
    roots = np.roots(np.polysub(p1, p2))
    roots = roots[np.isreal(roots)].real
    lo, hi = T[near].min(), T[near].max()
    if len(sign) == 0:   # extrapolated: the fit windows end at the grid edge
        lo, hi = lo - extrapolate * width, hi + extrapolate * width
    inside = roots[(roots >= lo - 1e-12) & (roots <= hi + 1e-12)]
    tc = float(inside[np.argmin(np.abs(inside - t0))]) if len(inside) else float(t0)
    d1, d2 = np.polyder(p1), np.polyder(p2)
    return tc, float(np.polyval(p1, tc)), float(np.polyval(d1, tc)), float(np.polyval(d2, tc))


def nu_from_slope_ratio(ratio, b=2.0):
    """nu from (d xi_bL/dT)/(d xi_L/dT) = b^(1 + 1/nu) at the crossing
    (Sec. IV, quotient method; the paper's pairs have b = 2)."""
    return 1.0 / (np.log(ratio) / np.log(b) - 1.0)


def eta_from_chi_ratio(ratio, b=2.0):
    """eta from chi_bL / chi_L = b^(2 - eta) at the crossing (Sec. IV)."""
    return 2.0 - np.log(ratio) / np.log(b)


def value_at(T, y, t, n_fit=4):
    """y at temperature t from a linear fit to the n_fit grid temperatures
    nearest to t (the fits used at the crossing)."""
    T = np.asarray(T, dtype=np.float64)
    near = np.sort(np.argsort(np.abs(T - t))[:n_fit])
    return float(np.polyval(np.polyfit(T[near], np.asarray(y, dtype=np.float64)[near], 1), t))


def crossing_jackknife(T, blocks1, blocks2, n_fit=4, order=1):
    """crossing() of the block means, with jackknife errors over blocks
    (blocks: (nb, n_T) arrays, e.g. xi/L per disorder sample or time block).
    Returns dict of (value, error) for T_cross, y_cross and the slope ratio
    slope2/slope1 (for xi/L curves, 2^(1+1/nu) needs the ratio of d xi/dT,
    i.e. twice this ratio when the second curve is at twice the size)."""
    b1 = np.asarray(blocks1, dtype=np.float64)
    b2 = np.asarray(blocks2, dtype=np.float64)

    def f(m):
        n = m.shape[0] // 2
        tc, yc, s1, s2 = crossing(T, m[:n], m[n:], n_fit, order)
        return np.array([tc, yc, s2 / s1])

    full, err = jackknife(np.concatenate([b1, b2], axis=1), f)
    return {"T_cross": (full[0], err[0]), "y_cross": (full[1], err[1]), "slope_ratio": (full[2], err[2])}
