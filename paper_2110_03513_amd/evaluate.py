"""Quality of fitted partial effects: the MISE of the simulation study.

Sec. 4.1 measures partial-effect estimation by the mean integrated squared
error between each learner's estimated function and the true effect,
integrated over the feature's range and averaged over the features.  Here
the estimated functions come from a callable (a fit's partial effects on the
GPU), the true ones from the input generator.  Both are centred by their
mean over the sample rows before they are compared: a P-spline learner
carries the constant in its unpenalised null space, so the split of the
intercept between f0 and the learners is not identified, and the generator
centres its effects the same way.
"""
from __future__ import annotations

import numpy as np

from . import datagen


def simpson(values: np.ndarray, lo: float, hi: float) -> float:
    """Composite Simpson rule on an odd number of equally spaced points."""
    g = values.shape[0]
    if g < 3 or g % 2 == 0:
        raise ValueError("Simpson's rule needs an odd number of points >= 3")
    w = np.ones(g)
    w[1:-1:2] = 4.0
    w[2:-1:2] = 2.0
    return float((hi - lo) / (3.0 * (g - 1)) * np.dot(w, values))


def integrated_squared_error(est, truth, sample: np.ndarray, grid: int = 2001) -> float:
    """Integral over [min(sample), max(sample)] of the squared difference of
    two functions, each centred by its mean over the sample points."""
    sample = np.asarray(sample, dtype=np.float64)
    lo, hi = float(sample.min()), float(sample.max())
    xs = np.linspace(lo, hi, grid)
    ce = float(np.mean(est(sample)))
    ct = float(np.mean(truth(sample)))
    d = (est(xs) - ce) - (truth(xs) - ct)
    return simpson(d * d, lo, hi)


def mise(prob: dict, partial_effect, features=None, grid: int = 2001) -> float:
    """MISE over numeric features (all of them by default): the mean over
    features of the integrated squared error between the estimated partial
    effect ``partial_effect(j, values)`` and the generating effect."""
    x = np.asarray(prob["x"])
    kind = np.asarray(prob["kind"])
    if features is None:
        features = [j for j in range(x.shape[1]) if kind[j] == datagen.PSPLINE]
    vals = [integrated_squared_error(lambda v, j=j: partial_effect(j, v),
                                     lambda v, j=j: datagen.true_effect(prob, j, v),
                                     x[:, j], grid)
            for j in features]
    return float(np.mean(vals))
