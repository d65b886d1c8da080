"""Hologram generation loops in FP64 (oracle; test infrastructure).

Follows, in order:
  * Background section: far field of a 100%-fill SLM = 2D DFT
    (Eqs. fouriertrans2d5c/d); Fresnel holograms add a quadratic phase term.
  * Algorithms section: quantisation = adapting the ideal aperture to the
    SLM's states; the "three freedoms" (amplitude, phase, scale).
  * Floating Points section: every image is scaled automatically.
  * Iterative Fourier Transform Algorithms section: Gerchberg-Saxton (GS),
    its weighted variant and Liu-Taghizadeh (LT).
  * Time-Averaged Algorithms section: OSPR and adaptive OSPR.

Readings where the paper is silent (each is restated in the design notes):
  * Target preparation: T is scaled so that sum T^2 = Nx Ny.  For binary
    phase (L = 2) the replay of a real +-1 hologram is centro-symmetric,
    |R(u)| = |R(-u)|, so T is first replaced by the closest symmetric
    intensity, T <- sqrt((T(u)^2 + T(-u)^2) / 2), -u taken about the centre.
  * GS order: f0 -> [R = forward(f); nmse; R' = T R/|R|; g = backward(R');
    f = P_L(g)] x K -> nmse of the final, projected field.  The initial
    field is an unquantised random phase (or a supplied field / levels).
  * LT: at iteration i the amplitude is constrained inside the centred
    square of radius r0 + (i-1) dr pixels and left free (R' = R) outside;
    nmse is still taken over the whole plane.
  * Region of interest (Background section: many applications care about
    part of the replay field only, and restricting the error metric to it
    adds freedom; Algorithms section: amplitude freedom where the replay is
    not controlled).  A GS problem may carry a mask M of controlled pixels.
    The target outside M is ignored: T <- prepare(T_raw * M).  The
    controlled region is M, or M united with its mirror image for binary
    phase and amplitude SLMs, whose replay is centro-symmetric (that is also
    where the symmetrised target can be nonzero).  Inside the region
    R' = T R/|R|; outside R' = R; the NMSE counts the region only.  Weighted
    GS and LT do not take a region.
  * Weighted GS (the paper names weighting only): a leaky log-domain
    integrator of the amplitude error,
      w_k = clamp(w_{k-1} * ratio / m_{k-1}, 1e-6, 1e6) ** GAMMA,
      ratio = max(T, EPS) / max(|R|, EPS),
    on the support Omega = {T > 0} (w unchanged elsewhere); m_{k-1} = mean
    of w_{k-1} over Omega (m_0 = mean of the initial weights);
    R' = w_k T R/|R|.  T and |R| have unit rms (Parseval), so EPS = 0.1 is
    relative to the mean replay level; flooring both sides keeps a
    consistent target a fixed point and bounds the ratio's sensitivity to
    rounding in |R| near speckle zeros.  GAMMA = 1 is the plain
    multiplicative rule, which diverges for binary phase; GAMMA = 0.7 keeps
    the weights bounded.
  * Fresnel: single-transform Fresnel with chirp
    Q[y][x] = exp(i pi p^2 ((x - Nx/2)^2 + (y - Ny/2)^2) / (lambda z));
    forward R = centre(DFT(f Q)), backward f = IDFT(uncentre(R)) conj(Q).
  * Amplitude-modulating SLMs (Background section, the binary and
    multi-level amplitude schemes): the SLM shows real transmissions
    k / (L - 1) (slm.project_amplitude).  A non-negative transmission always
    sends mean(f) sqrt(Nx Ny) into the zero-order pixel (the DC of the
    centred replay, index (Ny/2, Nx/2)), which no amplitude hologram can
    control; that pixel is therefore left free (R' = R there, the amplitude
    freedom of the Algorithms section) and out of the NMSE.  The replay of a
    real field is centro-symmetric, so the target is symmetrised for every L
    as for binary phase.  Liu-Taghizadeh and OSPR stay phase-only.
  * 16-bit field storage (Floating Points section: 16-, 32- and 64-bit
    builds, throughput about inversely proportional to the bits): the
    complex field is held between the two halves of each transform pair as
    two IEEE binary16 values, arithmetic stays at full precision.  The
    halves are the row transform (SLM plane -> rows transformed) and the
    column transform; the stored quantities are the unnormalised row DFT of
    the modulated SLM field and the unnormalised column inverse DFT of the
    constrained replay, each times a power of two (2^-floor(log2(n)/2), n
    the transform length) that keeps typical magnitudes near 1 and changes
    no mantissa.  forward16 / backward16 round there (round to nearest
    even, as a binary16 conversion does).
  * OSPR: subframe n draws a uniform random replay phase phi_n, takes the
    binary projection of IDFT(T_n e^{i phi_n}), accumulates |R_n|^2 and
    reports the NMSE of the running-average amplitude sqrt(A_n / n).
    Adaptive feedback (compensating the cumulative error): the next
    subframe asks for the intensity still missing after n+1 frames,
    T_{n+1}^2 = max(0, (n+1) T^2 - A_n).  No global scale is needed: the
    binary projection ignores the scale of T_{n+1}, and Parseval fixes
    mean(A_n) = n = n mean(T^2) exactly.
"""
import numpy as np

from . import dft as _dft
from . import philox as _ph
from . import slm as _slm
from . import metrics as _m

EPS = 1e-6          # OSPR intensity floor
WGS_EPS = 0.1       # weighted-GS amplitude floor (unit-rms units)
WGS_GAMMA = 0.7     # weighted-GS leak exponent
W_MIN = 1e-6
W_MAX = 1e6


def mirror(T):
    """T(-u) about the replay centre: index (N - i) mod N along each axis."""
    ny, nx = T.shape
    iy = (-np.arange(ny)) % ny
    ix = (-np.arange(nx)) % nx
    return T[np.ix_(iy, ix)]


def prepare_target(T_raw, L, amplitude=False):
    """Target preparation (automatic scaling; symmetrisation for binary phase
    and for every amplitude SLM, whose real field has a centro-symmetric
    replay)."""
    T = np.asarray(T_raw, dtype=np.float64)
    if np.any(~np.isfinite(T)) or np.any(T < 0):
        raise ValueError("target amplitude must be finite and non-negative")
    if L == 2 or amplitude:
        T = np.sqrt(0.5 * (T * T + mirror(T) ** 2))
    e = float(np.sum(T * T))
    if e <= 0.0:
        raise ValueError("target has zero energy")
    ny, nx = T.shape
    return T * np.sqrt(nx * ny / e)


def fresnel_chirp(ny, nx, wavelength, pitch, z):
    """Quadratic phase Q[y][x] on centred pixel coordinates; None = Fourier."""
    if z is None or not np.isfinite(z) or z <= 0:
        return None
    y = np.arange(ny, dtype=np.float64) - ny / 2
    x = np.arange(nx, dtype=np.float64) - nx / 2
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    ph = np.pi * pitch * pitch * r2 / (wavelength * z)
    return np.cos(ph) + 1j * np.sin(ph)


def forward(f, Q=None):
    """SLM plane -> centred replay plane."""
    f = np.asarray(f, dtype=np.complex128)
    if Q is not None:
        f = f * Q
    return _dft.centre(_dft.dft2(f))


def backward(Rc, Q=None):
    """Centred replay plane -> SLM plane (inverse of forward())."""
    g = _dft.idft2(_dft.uncentre(np.asarray(Rc, dtype=np.complex128)))
    if Q is not None:
        g = g * np.conj(Q)
    return g


def half_scale(n):
    """Power-of-two scale of a stored 16-bit field plane for length-n transforms."""
    return 2.0 ** -(int(np.log2(n)) // 2)


def store16(Z, scale):
    """Z as a 16-bit field plane holds it: each of (scale Re Z, scale Im Z)
    rounded to IEEE binary16 (round to nearest even), then unscaled."""
    Z = np.asarray(Z, dtype=np.complex128) * scale
    out = np.empty(Z.shape, dtype=np.complex128)  # parts set one by one: inf stays inf
    out.real = Z.real.astype(np.float16).astype(np.float64) / scale
    out.imag = Z.imag.astype(np.float16).astype(np.float64) / scale
    return out


def checker(ny, nx):
    """(-1)^(x+y): multiplying the SLM field by it centres the replay."""
    return np.where(((np.arange(ny)[:, None] + np.arange(nx)[None, :]) & 1) == 1, -1.0, 1.0)


def forward16(f, Q=None, store=store16):
    """forward() with the field stored as 16-bit values between the row and
    column halves: h = f Q (-1)^(x+y); Z = unnormalised row DFT of h, stored;
    R = the column DFT of Z, unitary overall (centred by the checker)."""
    f = np.asarray(f, dtype=np.complex128)
    ny, nx = f.shape
    h = (f * Q if Q is not None else f) * checker(ny, nx)
    Z = store(h @ (_dft.dft_matrix(nx, -1).T * np.sqrt(nx)), half_scale(nx))
    return _dft.dft_matrix(ny, -1) @ Z / np.sqrt(nx)


def backward16(Rc, Q=None, store=store16):
    """backward() with the field stored as 16-bit values between the column
    and row halves: Y = unnormalised column inverse DFT of Rc, stored;
    g = the row inverse DFT of Y (unitary overall) times (-1)^(x+y) conj(Q)."""
    Rc = np.asarray(Rc, dtype=np.complex128)
    ny, nx = Rc.shape
    Y = store((_dft.dft_matrix(ny, +1) * np.sqrt(ny)) @ Rc, half_scale(ny))
    g = Y @ _dft.dft_matrix(nx, +1).T / np.sqrt(ny) * checker(ny, nx)
    return g * np.conj(Q) if Q is not None else g


def _phase_of(R):
    A = np.abs(R)
    return np.where(A > 0, R / np.where(A > 0, A, 1.0), 1.0 + 0j), A


def fienup_error(T, A, exclude=None, region=None):
    """Unscaled replay error sum (|R| - T)^2, the quantity GS never increases
    (exclude: a pixel left free, e.g. an amplitude SLM's zero order; region:
    the controlled pixels, the others being free)."""
    d = (np.asarray(A, dtype=np.float64) - np.asarray(T, dtype=np.float64)) ** 2
    if exclude is not None:
        d[exclude] = 0.0
    if region is not None:
        d[~region] = 0.0
    return float(np.sum(d))


def zero_order(ny, nx):
    """Index of the zero-order (DC) pixel of the centred replay plane."""
    return (ny // 2, nx // 2)


def lt_window(ny, nx, r):
    """Liu-Taghizadeh target region of radius r pixels: the centred square
    |v - ny/2| <= r, |u - nx/2| <= r of the replay plane.  The Iterative
    Fourier Transform Algorithms section has LT target part of the replay
    field first and enlarge it every iteration; the paper gives neither the
    region's shape nor its growth, so both are a reading."""
    v = np.abs(np.arange(ny) - ny // 2)[:, None]
    u = np.abs(np.arange(nx) - nx // 2)[None, :]
    return (v <= r) & (u <= r)


def roi_region(roi, L, amplitude=False):
    """Controlled replay pixels of a region-of-interest mask: M, or M with its
    mirror image for binary phase and amplitude SLMs."""
    M = np.asarray(roi) != 0
    return M | mirror(M) if (L == 2 or amplitude) else M


def gs(T_raw, iters, L, seed=0, init_levels=None, init_field=None,
       weighted=False, weights=None, optics=None, batch_item=0, lt=None, amplitude=False, field16=False,
       roi=None):
    """Gerchberg-Saxton / weighted GS / Liu-Taghizadeh.  Returns a dict of final state.

    optics = (wavelength_m, pitch_m, z_m) selects a Fresnel hologram.
    lt = (r0, dr) selects Liu-Taghizadeh (GS only): iteration i = 1..K
    constrains the replay amplitude only inside lt_window(r0 + (i-1) dr)
    and leaves it free (R' = R) outside.
    amplitude selects an L-level amplitude SLM (GS or weighted GS).
    field16 holds the field as 16-bit values between transform halves
    (forward16 / backward16).
    roi: optional [ny][nx] mask of controlled replay pixels (plain GS only;
    see the region-of-interest reading above).
    Keys: field (f_K), levels (k_K or None), g (the last field before
    projection), replay (R_K), nmse (K+1), fienup (K+1), weights (w_K),
    m (mean of w_K on Omega), target (prepared T).
    """
    if amplitude and (L < 2 or lt is not None):
        raise ValueError("an amplitude SLM has L >= 2 levels and runs GS or weighted GS")
    region = None
    if roi is not None:
        if lt is not None or weighted:
            raise ValueError("a region of interest runs with plain GS")
        M = np.asarray(roi) != 0
        if M.shape != np.shape(T_raw):
            raise ValueError("roi and target differ in shape")
        T_raw = np.where(M, np.asarray(T_raw, dtype=np.float64), 0.0)
        region = roi_region(M, L, amplitude)
    T = prepare_target(T_raw, L, amplitude)
    ny, nx = T.shape
    dc = zero_order(ny, nx) if amplitude else None
    Q = fresnel_chirp(ny, nx, *optics) if optics is not None else None
    if init_field is not None:
        f = np.asarray(init_field, dtype=np.complex128)
    elif init_levels is not None:
        k0 = np.asarray(init_levels, dtype=np.int64)
        f = _slm.amplitude_value(k0, L) + 0j if amplitude else _slm.level_phasor(k0, L)
    else:
        f = np.exp(1j * _ph.phase_field(seed, _ph.TAG_INIT, ny, nx, batch_item))
    levels = None if init_levels is None else np.asarray(init_levels, np.int64)
    omega = T > 0
    w = np.ones_like(T) if weights is None else np.asarray(weights, dtype=np.float64).copy()
    m = float(np.mean(w[omega])) if np.any(omega) else 1.0
    nm, fe = [], []
    g = None
    if lt is not None and weighted:
        raise ValueError("Liu-Taghizadeh is a GS variant: weighted=False")
    for it in range(iters):
        st = _iterate(T, L, f, Q, weighted, w, m, None if lt is None else lt[0] + it * lt[1], amplitude, field16,
                      region)
        nm.append(_m.nmse(T, st["A"], dc, region))
        fe.append(fienup_error(T, st["A"], dc, region))
        g, f, levels = st["g"], st["field"], st["levels"]
        if weighted:
            w = st["weights"]
            m = float(np.mean(w[omega])) if np.any(omega) else 1.0
    R = forward16(f, Q) if field16 else forward(f, Q)
    A = np.abs(R)
    nm.append(_m.nmse(T, A, dc, region))
    fe.append(fienup_error(T, A, dc, region))
    return dict(field=f, levels=levels, g=g, replay=R, nmse=np.array(nm),
                fienup=np.array(fe), weights=w, m=m, target=T, region=region)


def ospr_target(T, A_prev, n, adaptive):
    """Replay amplitude T_n asked of subframe n >= 1 (Time-Averaged Algorithms
    section: adaptive OSPR feeds back the error accumulated so far).

    Reading: subframe n asks for the intensity still missing once it is
    added to the n - 1 subframes already shown, so that their average would
    equal the target: T_n^2 = max(0, n T^2 - A_{n-1}).  Plain OSPR (and the
    first subframe, A_0 = 0, of either) asks for T itself.
    """
    if adaptive and n > 1:
        return np.sqrt(np.maximum(0.0, n * T * T - A_prev))
    return np.asarray(T, dtype=np.float64)


def ospr_subframe(T, A_prev, n, adaptive, seed=0, batch_item=0):
    """Subframe n >= 1 of (adaptive) OSPR from the accumulated intensity A_{n-1}.

    T is the prepared target.  Returns (levels_n, g_n, A_n, nmse_n).
    """
    ny, nx = T.shape
    Tn = ospr_target(T, A_prev, n, adaptive)
    phi = _ph.phase_field(seed, _ph.TAG_OSPR + n, ny, nx, batch_item)
    g = backward(Tn * np.exp(1j * phi))
    h, k = _slm.project(g, 2)
    A = A_prev + np.abs(forward(h)) ** 2
    return k, g, A, _m.nmse(T, np.sqrt(A / n))


def gs_step(T, L, f_prev, weighted=False, w_prev=None, optics=None, lt_r=None, next_nmse=True, amplitude=False,
            field16=False):
    """One GS / weighted GS / Liu-Taghizadeh iteration from a given state.

    T is the PREPARED target (prepare_target), f_prev the SLM field f_{k-1}
    and, for weighted GS, w_prev the weights w_{k-1}; the lagged mean
    m_{k-1} is the mean of w_prev over Omega = {T > 0} (see gs()).  lt_r is
    the Liu-Taghizadeh square's radius for this iteration (None: no region).
    Returns a dict: replay (R_k = forward(f_{k-1}), before the constraint),
    g (backward of the constrained replay, before projection), field (f_k),
    levels (None for L = 0), weights (w_k or None), nmse (NMSE of R_k) and
    nmse_next (NMSE of the replay of f_k; None when next_nmse is False, which
    saves its transform).  amplitude: an L-level amplitude SLM (zero order
    free and out of the NMSE).
    """
    T = np.asarray(T, dtype=np.float64)
    ny, nx = T.shape
    dc = zero_order(ny, nx) if amplitude else None
    Q = fresnel_chirp(ny, nx, *optics) if optics is not None else None
    m = None
    if weighted:
        w_prev = np.asarray(w_prev, dtype=np.float64)
        omega = T > 0
        m = float(np.mean(w_prev[omega])) if np.any(omega) else 1.0
    st = _iterate(T, L, np.asarray(f_prev, dtype=np.complex128), Q, weighted, w_prev, m, lt_r, amplitude, field16)
    fwd = forward16 if field16 else forward
    return dict(replay=st["R"], g=st["g"], field=st["field"], levels=st["levels"],
                weights=st["weights"] if weighted else None, nmse=_m.nmse(T, st["A"], dc),
                nmse_next=_m.nmse(T, np.abs(fwd(st["field"], Q)), dc) if next_nmse else None)


def _iterate(T, L, f, Q, weighted, w, m, lt_r, amplitude=False, field16=False, region=None):
    """The body of one iteration (Iterative Fourier Transform Algorithms
    section): R = forward(f); replay constraint (GS: R' = T R/|R|, R = 0
    gives T; weighted GS: the weight update, then R' = w T R/|R|;
    Liu-Taghizadeh: R' = T R/|R| inside the square of radius lt_r, R' = R
    outside; a region of interest likewise keeps R' = R outside its region;
    an amplitude SLM keeps R' = R at the zero order);
    g = backward(R'); f_next = P_L(g) (phase) or the nearest transmission
    (amplitude).  m is the lagged mean m_{k-1} of the weights over Omega."""
    ny, nx = T.shape
    R = forward16(f, Q) if field16 else forward(f, Q)
    ph, A = _phase_of(R)
    if lt_r is not None:
        Rp = np.where(lt_window(ny, nx, lt_r), T * ph, R)
    elif weighted:
        ratio = np.maximum(T, WGS_EPS) / np.maximum(A, WGS_EPS)
        w = np.where(T > 0, np.clip(w * ratio / m, W_MIN, W_MAX) ** WGS_GAMMA, w)
        Rp = w * T * ph
    else:
        Rp = T * ph
    if region is not None:
        Rp = np.where(region, Rp, R)
    if amplitude:
        dc = zero_order(ny, nx)
        Rp[dc] = R[dc]
    g = backward16(Rp, Q) if field16 else backward(Rp, Q)
    f_next, levels = _slm.project_amplitude(g, L) if amplitude else _slm.project(g, L)
    return dict(R=R, A=A, g=g, field=f_next, levels=levels, weights=w)


def ospr(T_raw, subframes, adaptive, seed=0, batch_item=0):
    """OSPR / adaptive OSPR with binary phase subframes.

    Returns levels (subframes, Ny, Nx), nmse per subframe of the running
    time-averaged replay amplitude, and the accumulated intensity A_N.
    """
    T = prepare_target(T_raw, 2)
    A = np.zeros_like(T)
    levels, nm = [], []
    for n in range(1, subframes + 1):
        k, _, A, e = ospr_subframe(T, A, n, adaptive, seed, batch_item)
        levels.append(k)
        nm.append(e)
    return dict(levels=np.array(levels), nmse=np.array(nm), accum=A, target=T)


def fresnel_propagate(field, wavelength, pitch, z, direction):
    """+1: SLM -> centred replay; -1: centred replay -> SLM."""
    field = np.asarray(field, dtype=np.complex128)
    ny, nx = field.shape
    Q = fresnel_chirp(ny, nx, wavelength, pitch, z)
    return forward(field, Q) if direction > 0 else backward(field, Q)
