"""Acceptance rule of the finite-difference gradient checks (no method
arithmetic): the survey's bounds on directional derivatives."""
import sys

import numpy as np


def check_fd(preds, fdv, spread):
    """Adjoint directional derivatives against central differences: every
    direction within 5e-2 and the median within 1e-2 of the rms
    finite-difference slope.  Random unit directions project the gradient onto
    values of either sign, some near zero, so the error is measured on the
    scale of the slopes rather than on each slope."""
    preds, fdv, spread = map(np.array, (preds, fdv, spread))
    scale = np.sqrt(np.mean(fdv ** 2))
    err = np.abs(preds - fdv) / scale
    cos = preds @ fdv / np.linalg.norm(preds) / np.linalg.norm(fdv)
    print(f"errors / rms slope: median {np.median(err):.3e}, worst {err.max():.3e}, "
          f"FD spread / rms worst {np.max(spread) / scale:.3e}, cosine over directions {cos:.6f}",
          file=sys.stderr, flush=True)
    assert np.median(err) <= 1e-2 and err.max() <= 5e-2 and cos > 0.999
