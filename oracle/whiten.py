"""FP64 oracle: spectral whitening of an echo cube (Eq. 9, Sec. II-E).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definition: the power estimate of frequency bin f is the average over every
(ping, element) row of the cube of |X(f)|^2, X the discrete Fourier
transform of the row (N_s samples); its average over the bins is mean P^.
The gain is

    G(f) = h(1 / (gamma mean P^ + P^(f))),

with h the normalisation that makes the smallest attenuation 0 dB (G
divided by its maximum).

Readings where the paper is silent: P^ is estimated from the whole cube; G
is a power gain, applied to the spectrum of every row as the amplitude
factor sqrt(G(f)) before the inverse transform.
"""
from __future__ import annotations

import numpy as np


def whiten(echo, gamma: float):
    """Returns (whitened echo complex128 [P, E, N_s], power estimate P^ [N_s], gain G [N_s])."""
    e = np.asarray(echo, dtype=np.complex128)
    X = np.fft.fft(e, axis=-1)
    Phat = (np.abs(X) ** 2).reshape(-1, e.shape[-1]).mean(axis=0)
    G = 1.0 / (gamma * Phat.mean() + Phat)
    G = G / G.max()
    out = np.fft.ifft(X * np.sqrt(G)[None, None, :], axis=-1)
    return out, Phat, G
