"""Unitary 2D DFT pair written out as its definition (oracle; test infrastructure).

Background section, Eq. fouriertrans2d5c (forward) and Eq. fouriertrans2d5d
(inverse):

    F[v][u] = (Nx Ny)^(-1/2) sum_x sum_y f[y][x] exp(-2 pi i (u x / Nx + v y / Ny))
    f[y][x] = (Nx Ny)^(-1/2) sum_u sum_v F[v][u] exp(+2 pi i (u x / Nx + v y / Ny))

Arrays are indexed [row][column] = [y][x] in the SLM plane and [v][u] in the
replay plane.  The double sum factorises into a left product with the Ny x Ny
DFT matrix and a right product with the Nx x Nx DFT matrix; a matrix product
is the only library primitive used.  Matrix entries use an exact integer
reduction (u*x mod N) before the float64 cosine/sine so that large products do
not lose phase accuracy.

Replay-plane centring is a reading (the paper does not state it): replay
arrays handed to users have the zero frequency at (Ny/2, Nx/2), i.e.
R_c[v'][u'] = F[(v' - Ny/2) mod Ny][(u' - Nx/2) mod Nx].
"""
import numpy as np


def dft_matrix(n, sign=-1):
    """W[k][m] = n^(-1/2) exp(sign * 2 pi i (k m mod n) / n), complex128."""
    k = np.arange(n, dtype=np.int64)
    m = np.outer(k, k) % n
    ang = (2.0 * np.pi / n) * m.astype(np.float64)
    return (np.cos(ang) + sign * 1j * np.sin(ang)) / np.sqrt(n)


def dft2(f):
    """Forward unitary 2D DFT, Eq. fouriertrans2d5c (natural, uncentred order)."""
    f = np.asarray(f, dtype=np.complex128)
    ny, nx = f.shape
    return dft_matrix(ny, -1) @ f @ dft_matrix(nx, -1).T


def idft2(F):
    """Inverse unitary 2D DFT, Eq. fouriertrans2d5d (natural, uncentred order)."""
    F = np.asarray(F, dtype=np.complex128)
    ny, nx = F.shape
    return dft_matrix(ny, +1) @ F @ dft_matrix(nx, +1).T


def centre(F):
    """Move the zero frequency from (0, 0) to (Ny/2, Nx/2)."""
    ny, nx = F.shape
    return np.roll(np.roll(F, ny // 2, axis=0), nx // 2, axis=1)


def uncentre(Fc):
    """Inverse of centre(): move the zero frequency back to (0, 0)."""
    ny, nx = Fc.shape
    return np.roll(np.roll(Fc, -(ny // 2), axis=0), -(nx // 2), axis=1)


def dft2_direct(f):
    """Eq. fouriertrans2d5c as a literal quadruple loop; tiny inputs only."""
    f = np.asarray(f, dtype=np.complex128)
    ny, nx = f.shape
    F = np.zeros((ny, nx), dtype=np.complex128)
    for v in range(ny):
        for u in range(nx):
            acc = 0j
            for y in range(ny):
                for x in range(nx):
                    ph = -2.0 * np.pi * (((u * x) % nx) / nx + ((v * y) % ny) / ny)
                    acc += f[y, x] * complex(np.cos(ph), np.sin(ph))
            F[v, u] = acc / np.sqrt(nx * ny)
    return F
