"""Static structure factor of oracle states -- TEST INFRASTRUCTURE ONLY.

S_a(k) = <|sum_x a(x) exp(-i k.x)|^2> / N for a = drho, u_x, u_y, u_z, with
k = 2 pi (m_x/n_x, m_y/n_y, m_z/n_z), from FP64 populations of the oracle,
by the plain definition: numpy's complex FFT over every mode, each mode
binned by |k| into equal-width shells on [0, pi sqrt(d)], k = 0 excluded.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def fields(q, shape, f, rho0):
    """drho, u_x, u_y, u_z of populations f ((q, N) FP64), each shaped
    (nz, ny, nx)."""
    nx, ny, nz = (tuple(shape) + (1, 1))[:3]
    c, _ = lattice(q)
    rho = f.sum(axis=0)
    u = (c.T.astype(float) @ f) / rho
    return [a.reshape(nz, ny, nx) for a in (rho - rho0, u[0], u[1], u[2])]


class ShellAverager:
    def __init__(self, shape, nbins):
        nx, ny, nz = (tuple(shape) + (1, 1))[:3]
        self.n = nx * ny * nz
        self.nbins = nbins
        kz = 2 * np.pi * np.fft.fftfreq(nz)[:, None, None]
        ky = 2 * np.pi * np.fft.fftfreq(ny)[None, :, None]
        kx = 2 * np.pi * np.fft.fftfreq(nx)[None, None, :]
        k = np.sqrt(kx ** 2 + ky ** 2 + kz ** 2)
        d = sum(1 for s in (nx, ny, nz) if s > 1)
        kmax = np.pi * np.sqrt(d) * (1 + 1e-12)
        self.bin = np.minimum((k / kmax * nbins).astype(int), nbins - 1)
        self.bin[0, 0, 0] = -1
        self.k = k
        self.acc = np.zeros((4,) + k.shape)
        self.samples = 0

    def add(self, flds):
        for a, fld in enumerate(flds):
            self.acc[a] += np.abs(np.fft.fftn(fld)) ** 2 / self.n
        self.samples += 1

    def shells(self):
        out = np.zeros((self.nbins, 6))
        sel = self.bin >= 0
        b = self.bin[sel]
        cnt = np.bincount(b, minlength=self.nbins).astype(float)
        out[:, 1] = cnt
        with np.errstate(invalid="ignore", divide="ignore"):
            out[:, 0] = np.where(cnt > 0, np.bincount(b, self.k[sel], self.nbins) / cnt, 0.0)
            for a in range(4):
                s = np.bincount(b, self.acc[a][sel], self.nbins)
                out[:, 2 + a] = np.where(cnt > 0, s / cnt / max(self.samples, 1), 0.0)
        return out
