"""FP64 CPU oracle of the paper's phase-only hologram (POH) conversion
(Sec. 3.3) -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; it shares nothing with the GPU package.

Readings (the printed Smooth POH formula is garbled: it assigns the amplitude
itself to the even cells):
  * Smooth POH is the double-phase amplitude coding of Hsueh and Sawchuk
    (1978) as used by Maimone et al. (2017): per colour channel the amplitude
    is normalised by its maximum, A_n = |H| / max |H| (A_n = 0 if H = 0
    everywhere), and with phi = arg H the checkerboard takes
    phi + arccos(A_n) where the pixel's row + column is even and
    phi - arccos(A_n) where it is odd, so that the mean of two neighbouring
    phasors is A_n e^{j phi}.
  * L_extract of the Random POH sums its terms over planes; every squared
    norm and the complex L1 norm is read as a mean over the elements, as for
    L_recon (so the plane sum becomes a plane average, a constant factor).
    ||z||_{1,C} = |Re z| + |Im z| summed (here averaged) over elements.
"""
import numpy as np

from . import oracle as O

LAMBDA_COMP = 0.1
LAMBDA_FIELD = 0.01


def dpac(field):
    """Complex [C][H][W] -> double-phase POH phases [C][H][W]."""
    f = np.asarray(field, np.complex128)
    A = np.abs(f)
    amax = A.reshape(A.shape[0], -1).max(axis=1)
    An = np.where(amax[:, None, None] > 0, A / np.where(amax > 0, amax, 1.0)[:, None, None], 0.0)
    An = np.minimum(An, 1.0)
    phi = np.angle(f)
    H, W = f.shape[1:]
    even = ((np.arange(H)[:, None] + np.arange(W)[None, :]) % 2) == 0
    d = np.arccos(An)
    return np.where(even[None], phi + d, phi - d)


def recon_terms(u, target, mask):
    return O.mse(u, target) if mask is None else O.recon(u, target, mask)


def extract_loss(u, u_rand, target, mask=None, lc=LAMBDA_COMP, lf=LAMBDA_FIELD):
    """L_extract for the propagated fields u (of the Gaussians' hologram) and
    u_rand (of the random POH), [L][C][H][W].  Returns (loss, dL/du, dL/du_rand)
    with dL/du = dL/dRe(u) + j dL/dIm(u)."""
    u = np.asarray(u, np.complex128)
    ur = np.asarray(u_rand, np.complex128)
    l1, I, g1 = recon_terms(u, target, mask)
    l2, Ir, g2 = recon_terms(ur, target, mask)
    n = I.size
    dI = I - Ir
    d = u - ur
    loss = l1 + l2 + lc * float(np.sum(dI * dI) / n) + lf * float(np.sum(np.abs(d.real) + np.abs(d.imag)) / n)
    gc = 2.0 * lc * dI / n            # d/dI of the comparison term (and -d/dI_rand)
    gf = lf * (np.sign(d.real) + 1j * np.sign(d.imag)) / n
    gu = g1 + gc * 2.0 * u + gf
    gur = g2 - gc * 2.0 * ur - gf
    return loss, gu, gur


def phase_grad(phase, grad_field):
    """dL/dphi for H = exp(j phi) from g = dL/dRe(H) + j dL/dIm(H): Im(conj(H) g)."""
    H = np.exp(1j * np.asarray(phase, np.float64))
    return np.imag(np.conj(H) * np.asarray(grad_field, np.complex128))
