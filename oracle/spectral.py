"""FP64 cFSE carried out on spectra (Section III, eqs. (11), (12), (13),
(15), (18)).

TEST INFRASTRUCTURE ONLY: used by tests/ and the benchmark's CPU reference
leg; never by the product path. Shares no code with the GPU side.

Section III shows that the spatial residual never has to be formed: the
projection of the weighted residual onto every basis function (the
numerator of eq. (9)) is the DFT of w*r, and subtracting c*phi_(u,v) from r
changes that DFT by c times the window's DFT moved cyclically by (u, v)
(eq. (18)). This module keeps exactly that state, the *residual spectrum*,
as an F x F complex array, and advances it one selection at a time:

* start: residual spectrum = DFT(s*w), window spectrum = DFT(w) on the
  zero-padded F x F grid (eq. (11)); the estimation constant is
  gamma / DFT(w)[0, 0], because DFT(w)[0, 0] = sum(w) is the denominator of
  eq. (9) for every bin;
* selection: the bin of largest squared magnitude of the residual spectrum
  (eq. (12)), lowest linear index k*F + l among bins within a relative
  1e-12 of the largest (real input makes conjugate bins tie exactly);
* estimate: c = gamma * residual_spectrum[u, v] / sum(w) (eq. (13));
* update: residual_spectrum[k, l] -= c * window_spectrum[(k-u) % F, (l-v) % F]
  for every bin (eq. (18));
* the model is the list of (bin, c) terms; eq. (15) says its F x F
  coefficient map holds F*F*c per term, whose inverse DFT is the model, so
  on the area the model is sum c * exp(+j2pi(u m + v n)/F), evaluated here
  with two synthesis matrices.

It is a pin for the direct-projection oracle (each spectral state must
equal the projection of the spatial residual of eq. (17)) and the FP64 CPU
speed reference of the method in its frequency-domain form.
"""
import numpy as np

TIE_RTOL = 1e-12


class SpectralState:
    """Residual spectrum of one area and the terms chosen so far."""

    def __init__(self, s, w, F, gamma):
        M, N = s.shape
        if F < M or F < N:
            raise ValueError("transform smaller than the area")
        grid = np.zeros((F, F), dtype=np.complex128)
        grid[:M, :N] = s * w
        self.residual = np.fft.fft2(grid)                 # eq. (11), DFT(s*w)
        grid[:] = 0
        grid[:M, :N] = w
        self.window = np.fft.fft2(grid)                   # eq. (11), DFT(w)
        total = self.window[0, 0].real                    # sum of the weights
        if not total > 0:
            raise ValueError("empty support area (sum of weights is zero)")
        self.F, self.shape = F, (M, N)
        self.scale = gamma / total                        # eq. (13) without a division per step
        self._rows = np.arange(F)
        self.terms = []                                   # (linear bin, c)

    def strongest(self):
        """eq. (12): linear index of the largest |residual spectrum|^2."""
        p = (self.residual.real ** 2 + self.residual.imag ** 2).ravel()
        return int(np.flatnonzero(p >= p.max() * (1.0 - TIE_RTOL))[0])

    def advance(self, idx=None):
        """One selection (given or by eq. (12)), estimate (eq. (13)) and
        spectral update (eq. (18)); returns (idx, c)."""
        if idx is None:
            idx = self.strongest()
        u, v = divmod(int(idx), self.F)
        c = self.scale * self.residual[u, v]
        ks = (self._rows - u) % self.F
        ls = (self._rows - v) % self.F
        self.residual -= c * self.window[np.ix_(ks, ls)]
        self.terms.append((int(idx), complex(c)))
        return int(idx), complex(c)

    def model(self):
        """Complex model on the M x N area: sum over terms of
        c * exp(+j2pi(u m + v n)/F) (eq. (15) brought back to space)."""
        M, N = self.shape
        F = self.F
        coef = np.zeros((F, F), dtype=np.complex128)
        for idx, c in self.terms:
            coef[divmod(idx, F)] += c
        up = np.exp(2j * np.pi * np.outer(np.arange(M), np.arange(F)) / F)    # M x F
        across = np.exp(2j * np.pi * np.outer(np.arange(F), np.arange(N)) / F)  # F x N
        return up @ coef @ across


def run(s, w, F, gamma, iters, forced=None):
    """``iters`` steps from the start state; ``forced`` optionally gives the
    bin of every step. Returns (bins, coefficients, complex model on the
    area)."""
    st = SpectralState(s, w, F, gamma)
    for nu in range(iters):
        st.advance(None if forced is None else forced[nu])
    bins = [i for i, _ in st.terms]
    coefs = [c for _, c in st.terms]
    return bins, coefs, st.model()
