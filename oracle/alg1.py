"""FP64 frequency-domain cFSE, following Algorithm 1 of the paper.

TEST INFRASTRUCTURE ONLY: used by tests/ and the benchmark's CPU-baseline
leg; never by the product path. Shares no code with the GPU side.

Where ``oracle.cfse`` re-projects the spatial residual every iteration, this
module does what Section III derives: transform s*w and w once (eq. (11)),
select by the largest |R_w|^2 (eq. (12)), estimate c = gamma*R_w[u,v]/W[0,0]
(eq. (13)), add F*F*c to one model bin (eq. (15)) and subtract c times the
cyclically shifted window spectrum from every bin (eq. (18)); the model is
brought back with one inverse transform and its real part fills B.

It is a pin for the direct-projection oracle (eq. (18) must reproduce
eq. (17) followed by eq. (7)) and the fair FP64 CPU speed reference.
The transform size F plays the role of M x N in eqs. (15), (16).
"""
import numpy as np

TIE_RTOL = 1e-12


def _pick(mag2, forced, nu):
    if forced is not None:
        return int(forced[nu])
    c = mag2.ravel()
    return int(np.flatnonzero(c >= c.max() * (1.0 - TIE_RTOL))[0])


def cfse_fft(s, w, F, gamma, iters, forced=None):
    """Algorithm 1 on an M x N area zero-padded to F x F. Returns
    (seq, chat, g) with g the complex model on the area."""
    M, N = s.shape
    x = np.zeros((F, F), dtype=np.complex128)
    x[:M, :N] = s * w
    wp = np.zeros((F, F))
    wp[:M, :N] = w
    Rw = np.fft.fft2(x)                       # R_w = FFT{s w}
    Wf = np.fft.fft2(wp)                      # W = FFT{w}
    W0bar = 1.0 / Wf[0, 0].real               # 1 / W[0,0]
    G = np.zeros((F, F), dtype=np.complex128)
    seq, chat = [], []
    for nu in range(iters):
        idx = _pick(np.abs(Rw) ** 2, forced, nu)
        u, v = divmod(idx, F)
        c = gamma * Rw[u, v] * W0bar          # eq. (13)
        G[u, v] += F * F * c                  # eq. (15)
        Rw = Rw - c * np.roll(Wf, (u, v), axis=(0, 1))   # eq. (18): W[k-u, l-v]
        seq.append(idx)
        chat.append(complex(c))
    g = np.fft.ifft2(G)[:M, :N]
    return seq, chat, g
