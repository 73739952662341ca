"""Vibrational and polariton spectra from recorded MD trajectories.

Host-side post-processing of series sampled once per MD step (the device path
records them; nothing here runs on the GPU).  The spectrum is the dipole
(or photon-coordinate) autocorrelation transformed with an omega^2 prefactor
(Results: I(omega) proportional to omega^2 times the windowed cosine transform
of C(t), C the time-origin averaged autocorrelation).  The paper's smoothing is
a weighted moving average; the reading taken here is a Hann window over lags up
to half the run, zero padding by 8 and the peak located by a parabola through
the largest sample and its two neighbours.  The same processing is applied to
every path that is compared, so its small bias cancels in peak shifts.
"""
import numpy as np

HARTREE_CM = 219474.6313632  # 1 hartree in cm^-1 (angular frequency in a.u. -> wavenumber)


def autocorrelation(x, max_lag=None):
    """C(t) = < dx(t0 + t) dx(t0) >, averaged over time origins t0 and over the
    series, for x of shape [T] or [T, K] (T samples of K series) with each series'
    time mean removed (dx = x - <x>).  Lags 0..max_lag (default T // 2); the
    average over origins divides by the T - t pairs of each lag."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T = x.shape[0]
    L = T // 2 if max_lag is None else int(max_lag)
    if not 0 < L < T:
        raise ValueError("need 0 < max_lag < number of samples")
    dx = x - x.mean(axis=0)
    nfft = 1 << int(np.ceil(np.log2(2 * T)))  # zero padding: linear, not circular, correlation
    f = np.fft.rfft(dx, n=nfft, axis=0)
    s = np.fft.irfft(f * np.conj(f), n=nfft, axis=0)[: L + 1]
    s /= (T - np.arange(L + 1))[:, None]
    return s.mean(axis=1)


def spectrum(C, dt, pad=8, omega_squared=True):
    """I(omega) = omega^2 [w_0 C_0 + 2 sum_{t=1..L} w_t C_t cos(omega t dt)] with the
    half Hann window w_t = (1 + cos(pi t / L)) / 2 over the L + 1 lags of C, on a
    grid refined by zero padding the even extension to pad * 2L points.
    Returns (wavenumbers in cm^-1, I); dt is the sampling interval in atomic
    units of time (omega in hartree)."""
    C = np.asarray(C, dtype=np.float64)
    L = len(C) - 1
    if L < 2:
        raise ValueError("need at least three lags")
    w = 0.5 * (1.0 + np.cos(np.pi * np.arange(L + 1) / L))
    n = pad * 2 * L
    y = np.zeros(n)
    y[: L + 1] = w * C
    y[n - L:] = (w * C)[1:][::-1]
    S = np.fft.rfft(y).real  # w_0 C_0 + 2 sum_t w_t C_t cos(2 pi k t / n)
    omega = 2.0 * np.pi * np.arange(len(S)) / (n * dt)
    I = omega ** 2 * S if omega_squared else S
    return omega * HARTREE_CM, I


def peak(freq, I, lo, hi):
    """Position of the largest value of I with lo <= freq <= hi, refined by the
    parabola through that sample and its neighbours (the sample itself when it
    sits on the edge of the grid)."""
    freq = np.asarray(freq)
    I = np.asarray(I)
    idx = np.nonzero((freq >= lo) & (freq <= hi))[0]
    if len(idx) == 0:
        raise ValueError("no frequencies in the band")
    k = idx[np.argmax(I[idx])]
    if k == 0 or k == len(I) - 1:
        return float(freq[k])
    a, b, c = I[k - 1], I[k], I[k + 1]
    den = a - 2.0 * b + c
    d = 0.5 * (a - c) / den if den != 0.0 else 0.0
    return float(freq[k] + d * (freq[k + 1] - freq[k]))


def centroid(freq, I, lo, hi):
    """First moment sum(f I) / sum(I) of the spectrum over lo <= freq <= hi (a
    band position that does not jump between neighbouring maxima of a broad,
    noisy band the way the largest value can)."""
    freq = np.asarray(freq)
    I = np.asarray(I)
    m = (freq >= lo) & (freq <= hi)
    if not np.any(m):
        raise ValueError("no frequencies in the band")
    w = I[m]
    return float(np.sum(freq[m] * w) / np.sum(w))


def overlap(freq, Ia, Ib, lo, hi):
    """Normalised overlap sum(Ia Ib) / sqrt(sum(Ia^2) sum(Ib^2)) of two spectra on
    the same grid over lo <= freq <= hi: 1 for spectra of the same shape, whatever
    their scale; it weighs the whole band, not only its largest line."""
    freq = np.asarray(freq)
    m = (freq >= lo) & (freq <= hi)
    if not np.any(m):
        raise ValueError("no frequencies in the band")
    a, b = np.asarray(Ia)[m], np.asarray(Ib)[m]
    return float(np.sum(a * b) / np.sqrt(np.sum(a * a) * np.sum(b * b)))


def resolution_cm(n_samples, dt):
    """Frequency resolution 2 pi / (T dt) of a run of n_samples steps, in cm^-1."""
    return 2.0 * np.pi / (n_samples * dt) * HARTREE_CM


def report_from_acf(Ca, Cb, dt, lo, hi, n_samples):
    """Peak and band-centroid positions of two runs from their (averaged)
    autocorrelations: the largest peak in [lo, hi] cm^-1 of each, and the first
    moment of each spectrum over that same fixed band (it depends on neither
    run; a peak can jump between neighbouring maxima of a broad noisy band, the
    centroid cannot); the two strongest lines of each (top_peaks), the shift
    of run a's line nearest to run b's largest value, and the normalised
    overlap of the two spectra over the band.  The resolution
    2 pi / (n_samples dt) is returned beside them; no position is meaningful to
    much better than a fraction of it."""
    fa, Ia = spectrum(Ca, dt)
    fb, Ib = spectrum(Cb, dt)
    pa, pb = peak(fa, Ia, lo, hi), peak(fb, Ib, lo, hi)
    ca, cb = centroid(fa, Ia, lo, hi), centroid(fb, Ib, lo, hi)
    la, lb = top_peaks(fa, Ia, lo, hi), top_peaks(fb, Ib, lo, hi)
    # the line of run a nearest to run b's largest value: the same line of the
    # band followed across the runs, where their largest values can sit on
    # different lines of a multi-line band
    near = min(la, key=lambda f: abs(f - pb)) if la else None
    return {"peak_a_cm": pa, "peak_b_cm": pb, "shift_cm": pa - pb,
            "matched_line_shift_cm": (near - pb) if near is not None else None,
            "centroid_a_cm": ca, "centroid_b_cm": cb, "centroid_shift_cm": ca - cb,
            "lines_a_cm": la, "lines_b_cm": lb,
            "overlap": overlap(fa, Ia, Ib, lo, hi),
            "band_cm": [lo, hi], "resolution_cm": resolution_cm(n_samples, dt)}


def peak_report(series_a, series_b, dt, lo, hi):
    """report_from_acf for two runs recorded from the same start (series [T, K],
    the autocorrelation averaged over the K series)."""
    return report_from_acf(autocorrelation(series_a), autocorrelation(series_b), dt, lo, hi, len(series_a))


def spectrum_per_series(x, dt, pad=8, omega_squared=True):
    """Spectrum of each column of x [T, K] separately (e.g. the angle-resolved
    photon spectra I_k(omega), one column per k).  Returns (wavenumbers, I [K, F])."""
    x = np.asarray(x, dtype=np.float64)
    out = []
    freq = None
    for k in range(x.shape[1]):
        freq, I = spectrum(autocorrelation(x[:, k]), dt, pad=pad, omega_squared=omega_squared)
        out.append(I)
    return freq, np.array(out)


def averaged_spectrum(x, dt, columns, pad=8, omega_squared=False):
    """One spectrum from the time-origin autocorrelations of the selected
    columns of x [T, K], averaged over those columns (e.g. the photon
    coordinates q_k of all modes near normal incidence, whose frequencies
    differ by less than the resolution).  Returns (wavenumbers, I)."""
    x = np.asarray(x, dtype=np.float64)
    cols = np.asarray(columns)
    if cols.size == 0:
        raise ValueError("no columns selected")
    return spectrum(autocorrelation(x[:, cols]), dt, pad=pad, omega_squared=omega_squared)


def top_peaks(freq, I, lo, hi, count=2, rel=0.1):
    """The `count` highest local maxima of I with lo <= freq <= hi and at least
    rel times the largest value there (the Hann window's side lobes stay below
    3 % of their line), each refined by a parabola through its neighbours, in
    increasing frequency."""
    freq = np.asarray(freq)
    I = np.asarray(I)
    idx = np.nonzero((freq >= lo) & (freq <= hi))[0]
    idx = idx[(idx > 0) & (idx < len(I) - 1)]
    if len(idx) == 0:
        return []
    floor = rel * np.max(I[idx])
    loc = [k for k in idx if I[k] >= I[k - 1] and I[k] > I[k + 1] and I[k] >= floor]
    loc = sorted(loc, key=lambda k: -I[k])[:count]
    out = []
    for k in loc:
        a, b, c = I[k - 1], I[k], I[k + 1]
        den = a - 2.0 * b + c
        d = 0.5 * (a - c) / den if den != 0.0 else 0.0
        out.append(float(freq[k] + d * (freq[k + 1] - freq[k])))
    return sorted(out)
