"""RIS configuration for the paper's scenario (test helper).

Section III configures the on/off elements (amplitude 1.25) with an
algorithm of another paper that this one does not give; the stand-in here
maximises the received field at one point exactly over on/off choices of
the form "on iff the element's channel lies within 90 degrees of a
reference phase", the optimal family for maximising |sum of the selected
terms| (scanned over 720 reference phases).
"""
import math

import numpy as np


def configure_on_off(h: np.ndarray, amp: float = 1.25) -> np.ndarray:
    best, choice = -1.0, None
    for ph in np.linspace(0.0, 2.0 * math.pi, 720, endpoint=False):
        sel = np.cos(np.angle(h) - ph) > 0.0
        v = abs(h[sel].sum())
        if v > best:
            best, choice = v, sel
    return np.where(choice, amp, 0.0).astype(np.complex128)


def small_scale_period(P: np.ndarray, spacing: float, longest: float = 0.05) -> float:
    """Dominant spatial period of a sampled map below ``longest`` (the beam's
    large-scale envelope excluded): peak of the 2-D spectrum of P - mean."""
    ny, nx = P.shape
    F = np.abs(np.fft.fft2(P - P.mean()))
    fx = np.fft.fftfreq(nx, d=spacing)[None, :]
    fy = np.fft.fftfreq(ny, d=spacing)[:, None]
    k = np.hypot(fx, fy)
    F[k < 1.0 / longest] = 0.0
    iy, ix = np.unravel_index(np.argmax(F), F.shape)
    return 1.0 / k[iy, ix]
