"""FP64 oracle: range compression and basebanding of an echo cube (the
matched filter with the transmitted waveform q of Eq. 1, Sec. II-A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. 1 models each received time series as a sum of copies of q delayed by the
two-way travel time; the backprojection sum reads a range-compressed complex
baseband echo, whose point response peaks at that delay. This step produces
it from the received signal.

Definition, per (ping, element) row x[k], k < N_s, sampled at
t_k = t0 + k / f_s:

    baseband:  b[k] = x[k] exp(-j 2 pi f_c t_k)           (when mix is set)
    compress:  y[n] = (1 / sum_m |q[m]|^2) sum_{m<M} b[n + m] conj(q[m]),

with b[k] = 0 for k >= N_s (the record ends) and q[m], m < M, the waveform's
complex baseband samples at f_s from the start of transmission.

Readings where the paper is silent: the received samples are the analytic
(complex) signal, sampled at f_s (bandpass sampling, so basebanding is the
exact complex mix above and needs no filter); a row already at baseband
skips the mix; the filter is normalised by the replica's energy, so a
delayed copy of q compresses to a peak of exactly one at its delay; the
output keeps the input's N_s samples.
"""
from __future__ import annotations

import numpy as np


def range_compress(echo, replica, f_c: float, f_s: float, t0: float, mix: bool = True):
    """Returns the range-compressed baseband echo, complex128 of the input's shape [..., N_s]."""
    x = np.asarray(echo, dtype=np.complex128)
    q = np.asarray(replica, dtype=np.complex128).reshape(-1)
    Ns, M = x.shape[-1], q.shape[0]
    b = x
    if mix:
        t = t0 + np.arange(Ns, dtype=np.float64) / f_s
        b = x * np.exp(-2j * np.pi * f_c * t)
    energy = np.sum(np.abs(q) ** 2)
    rows = b.reshape(-1, Ns)
    out = np.empty_like(rows)
    for r in range(rows.shape[0]):
        padded = np.concatenate([rows[r], np.zeros(M - 1, dtype=np.complex128)])
        # numpy's correlate gives c[n] = sum_m padded[n + m] conj(q[m]), n < N_s
        out[r] = np.correlate(padded, q, mode="valid")
    return (out / energy).reshape(x.shape)
