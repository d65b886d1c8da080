"""Error metrics (oracle; test infrastructure).

Error Metrics section, Eq. mse: the mean squared error between target and
replay amplitudes,

    E_MSE(T, R) = 1/(Nx Ny) sum_x sum_y (|T| - |R|)^2 .

Algorithms section ("three freedoms"): scale is one of the freedoms, so the
replay is compared after the best uniform scale.  Reading (the paper names
no normalised metric): NMSE is the MSE at the least-squares optimal scale s,
normalised by the target energy,

    NMSE(T, A) = min_s sum (T - s A)^2 / sum T^2
               = 1 - (sum T A)^2 / (sum T^2 * sum A^2)

over the whole replay plane, with s = sum T A / sum A^2.  For an
amplitude-modulating SLM the zero-order pixel is left out (see hologram).
Background section: many applications care about part of the replay field
only, and the error metric may then count that region alone; with a region
R the sums run over R (T and A taken as zero elsewhere).
"""
import numpy as np


def mse(T, R):
    """Eq. mse, literally."""
    T = np.asarray(T)
    R = np.asarray(R)
    ny, nx = T.shape
    return float(np.sum((np.abs(T) - np.abs(R)) ** 2) / (nx * ny))


def nmse(T, A, exclude=None, region=None):
    """Scale-optimal normalised MSE of replay amplitude A against target T;
    exclude: optional (row, column) of one pixel left out of the sums;
    region: optional boolean mask, the only pixels counted."""
    T = np.array(T, dtype=np.float64)
    A = np.array(A, dtype=np.float64)
    if exclude is not None:
        T[exclude] = 0.0
        A[exclude] = 0.0
    if region is not None:
        T[~region] = 0.0
        A[~region] = 0.0
    sta = float(np.sum(T * A))
    saa = float(np.sum(A * A))
    stt = float(np.sum(T * T))
    if saa == 0.0 or stt == 0.0:
        return 1.0
    return 1.0 - sta * sta / (stt * saa)
