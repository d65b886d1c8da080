"""SLM constraint: projection onto the SLM's phase set (oracle; test infrastructure).

Algorithms section: the ideal aperture must be adapted ("quantised") to what
the SLM can display.  Example section, Listing 1 (quantiseDiscretePhase):
take the argument of the field, snap it to the nearest of the SLM's uniform
levels and return a unit phasor at that level.

Reading used here: full-circle uniform levels 2 pi k / L, k = 0..L-1 (the
listing with minimum 0 and maximum 2 pi (L-1)/L, spacing 2 pi / L).  The
index is k = floor(theta L / (2 pi) + 1/2) mod L with theta = atan2(Im, Re)
in (-pi, pi].  The listing rounds half away from zero; the two rules only
differ at exact ties, which parity treats as exempt.  L = 2 is binary phase
{0, pi}; L = 0 means continuous phase g/|g| (g = 0 maps to 1).

Amplitude-modulating SLMs (Background section: binary and multi-level
amplitude schemes; the listing's nearest-neighbour rule applied to the
transmission instead of the phase).  Reading: L uniform transmissions
a_k = k / (L - 1) in [0, 1] (binary: {0, 1}); the displayed field is real, so
the nearest a_k to a complex g in the Euclidean sense is the nearest to
Re g, k = clamp(floor(Re(g) (L - 1) + 1/2), 0, L - 1).  The field g is taken
at the scale of the unit-rms target (unitary transforms), with no further
normalisation.
"""
import numpy as np


def level_index(g, L):
    """Nearest uniform phase level index k in [0, L) for each complex g."""
    theta = np.arctan2(np.imag(g), np.real(g))
    return np.mod(np.floor(theta * L / (2.0 * np.pi) + 0.5), L).astype(np.int64)


def level_phasor(k, L):
    """Unit phasor exp(2 pi i k / L), evaluated with an exact k mod L reduction."""
    ang = 2.0 * np.pi * (np.mod(k, L).astype(np.float64) / L)
    return np.cos(ang) + 1j * np.sin(ang)


def project(g, L):
    """P_L(g): returns (unit-modulus field, level indices or None for L = 0)."""
    g = np.asarray(g, dtype=np.complex128)
    if L == 0:
        a = np.abs(g)
        out = np.where(a > 0, g / np.where(a > 0, a, 1.0), 1.0 + 0j)
        return out, None
    k = level_index(g, L)
    return level_phasor(k, L), k


def boundary_margin(g, L):
    """Angular distance (rad) from arg g to the nearest decision boundary of P_L.

    Boundaries sit at (2m + 1) pi / L.  Pixels with g = 0 get margin 0.
    Parity treats level mismatches with margin below 1e-5 rad as exempt.
    """
    theta = np.arctan2(np.imag(g), np.real(g))
    half = np.pi / L
    x = np.mod(theta + half, 2.0 * half)  # position inside the decision cell
    m = np.minimum(x, 2.0 * half - x)
    return np.where(np.abs(g) > 0, m, 0.0)


def amplitude_index(g, L):
    """Nearest transmission level index k in [0, L) of an amplitude SLM."""
    x = np.real(np.asarray(g, dtype=np.complex128)) * (L - 1)
    return np.clip(np.floor(x + 0.5), 0, L - 1).astype(np.int64)


def amplitude_value(k, L):
    """Transmission k / (L - 1) of level k of an L-level amplitude SLM."""
    return np.asarray(k, dtype=np.float64) / (L - 1)


def project_amplitude(g, L):
    """Projection onto an L-level amplitude SLM: (real field as complex, levels)."""
    k = amplitude_index(g, L)
    return amplitude_value(k, L) + 0j, k


def amplitude_margin(g, L):
    """Distance (in field units) from Re g to the nearest decision boundary
    (m + 1/2) / (L - 1), m = 0 .. L - 2, of the amplitude projection."""
    x = np.real(np.asarray(g, dtype=np.complex128)) * (L - 1)
    m = np.clip(np.floor(x), 0, L - 2)  # the boundary m + 1/2 below or above x is the nearest
    return np.abs(x - (m + 0.5)) / (L - 1)
