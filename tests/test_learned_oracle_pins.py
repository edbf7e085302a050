"""Closed-form pins of the learned-preconditioner oracle (oracle/learned.py): the Adam
step and the per-camera features.

These are values fixed by the definitions themselves, worked by hand:
  - Adam: with zero moments, the first step moves every parameter by
    lr * g / (|g| + eps), i.e. lr * sign(g) when |g| >> eps; a constant gradient keeps
    the bias-corrected moments exactly at g and g^2, so every later step is the same;
    two steps with gradients 1 and -3 have m^ = -21/19 and v^ = 9999/1999 after the
    second; at |g| = eps the first step is lr / 2.
  - Features: a diagonal block has zero correlations and centred log scales; a block
    with two known off-diagonal correlations puts them at their row-major
    upper-triangle positions; degree and lambda enter as log(1 + degree) and log lambda.

Each pin is a function of the oracle module, so the same checks also run on copies of
the oracle with one planted mistake (wrong bias correction, eps inside the square
root, transposed triangle order, uncentred log scales), each of which must fail.
"""
import math
import os
import types

import numpy as np
import pytest

from oracle import learned as L_real

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "learned.py")
LR = 1e-3


def _weights(mod, value):
    return mod.Weights.from_flat(np.full(mod.n_params(), float(value)))


def _step(mod, w, g, m, v, t):
    return mod.adam_step(w, g, m, v, t, lr=LR).flat()


def pin_adam_first_step_is_lr_sign(mod):
    rng = np.random.default_rng(11)
    p0 = rng.standard_normal(mod.n_params())
    gf = rng.choice([-1.0, 1.0], mod.n_params()) * 10.0 ** rng.uniform(-3, 1, mod.n_params())
    m = np.zeros(mod.n_params())
    v = np.zeros(mod.n_params())
    p1 = _step(mod, mod.Weights.from_flat(p0), mod.Weights.from_flat(gf), m, v, 1)
    # |g| >= 1e-3 so eps / |g| <= 1e-5
    return np.abs((p1 - p0) + LR * np.sign(gf)).max() <= LR * 1.1e-5


def pin_adam_constant_gradient(mod):
    """Bias-corrected moments of a constant gradient are exact: every step is lr * sign(g)."""
    w = _weights(mod, 0.25)
    g = _weights(mod, -0.7)
    m = np.zeros(mod.n_params())
    v = np.zeros(mod.n_params())
    p = w.flat()
    for t in range(1, 6):
        q = _step(mod, mod.Weights.from_flat(p), g, m, v, t)
        if np.abs((q - p) - LR).max() > LR * 1e-6:
            return False
        p = q
    return True


def pin_adam_two_steps_by_hand(mod):
    """g1 = 1, g2 = -3: m2 = 0.9 * 0.1 - 0.3 = -0.21, m^2 = -0.21 / 0.19 = -21/19;
    v2 = 0.999 * 0.001 + 0.009 = 0.009999, v^2 = 0.009999 / 0.001999 = 9999/1999."""
    m = np.zeros(mod.n_params())
    v = np.zeros(mod.n_params())
    p0 = 0.5
    p1 = _step(mod, _weights(mod, p0), _weights(mod, 1.0), m, v, 1)
    p2 = _step(mod, mod.Weights.from_flat(p1), _weights(mod, -3.0), m, v, 2)
    step1 = -LR * 1.0 / (1.0 + 1e-8)
    step2 = -LR * (-21.0 / 19.0) / (math.sqrt(9999.0 / 1999.0) + 1e-8)
    return (np.abs(p1 - (p0 + step1)).max() <= 1e-15 and
            np.abs(p2 - (p0 + step1 + step2)).max() <= 1e-15)


def pin_adam_eps_outside_root(mod):
    """|g| = eps on the first step: lr * eps / (eps + eps) = lr / 2."""
    m = np.zeros(mod.n_params())
    v = np.zeros(mod.n_params())
    p1 = _step(mod, _weights(mod, 0.0), _weights(mod, 1e-8), m, v, 1)
    return np.abs(p1 + LR / 2).max() <= LR * 1e-9


def pin_adam_zero_gradient_stays(mod):
    m = np.zeros(mod.n_params())
    v = np.zeros(mod.n_params())
    p1 = _step(mod, _weights(mod, 0.3), _weights(mod, 0.0), m, v, 1)
    return np.array_equal(p1, np.full(mod.n_params(), 0.3))


def pin_features_diagonal_block(mod):
    """D = diag(2^0, ..., 2^8): zero correlations, log scales (i - 4) ln 2."""
    D = np.diag(2.0 ** np.arange(9))[None]
    F = mod.features(D, np.array([0.0]), 1.0)[0]
    ok = np.abs(F[:36]).max() == 0.0
    ok &= np.abs(F[36:45] - (np.arange(9) - 4) * math.log(2.0)).max() <= 1e-15
    ok &= F[45] == 0.0 and F[46] == 0.0
    return bool(ok)


def pin_features_correlated_block(mod):
    """diag(1, 4, 9, 1, 1, 1, 1, 16, 1) with D[1,2] = 3 (correlation 3 / sqrt(4 * 9) = 0.5)
    and D[3,7] = -1 (correlation -1 / sqrt(1 * 16) = -0.25).  Row-major upper triangle
    without the diagonal: row i starts at 8 + 7 + ... (i terms), so (1,2) is entry 8 and
    (3,7) is entry 8 + 7 + 6 + 3 = 24."""
    d = np.array([1.0, 4.0, 9.0, 1.0, 1.0, 1.0, 1.0, 16.0, 1.0])
    D = np.diag(d)
    D[1, 2] = D[2, 1] = 3.0
    D[3, 7] = D[7, 3] = -1.0
    F = mod.features(D[None], np.array([3.0]), 1e-4)[0]
    want = np.zeros(36)
    want[8] = 0.5
    want[24] = -0.25
    ok = np.abs(F[:36] - want).max() <= 1e-15
    ld = np.log(d)
    ok &= np.abs(F[36:45] - (ld - ld.sum() / 9)).max() <= 1e-15
    ok &= abs(F[45] - math.log(4.0)) <= 1e-15
    ok &= abs(F[46] - math.log(1e-4)) <= 1e-15
    # lambda below the floor of the feature
    ok &= abs(mod.features(D[None], np.array([3.0]), 0.0)[0, 46] - math.log(1e-12)) <= 1e-15
    return bool(ok)


PINS = [pin_adam_first_step_is_lr_sign, pin_adam_constant_gradient, pin_adam_two_steps_by_hand,
        pin_adam_eps_outside_root, pin_adam_zero_gradient_stays, pin_features_diagonal_block,
        pin_features_correlated_block]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_passes(pin):
    assert pin(L_real)


def _mutant(old: str, new: str) -> types.ModuleType:
    src = open(SRC).read()
    assert src.count(old) == 1, old
    mod = types.ModuleType("learned_mutant")
    exec(compile(src.replace(old, new), "learned_mutant", "exec"), mod.__dict__)
    return mod


MUTANTS = {
    "no_bias_correction": ("mh = m / (1 - b1 ** t)", "mh = m"),
    "bias_correction_off_by_one": ("vh = v / (1 - b2 ** t)", "vh = v / (1 - b2 ** (t + 1))"),
    "eps_inside_root": ("np.sqrt(vh) + eps", "np.sqrt(vh + eps)"),
    "first_moment_weights_swapped": ("m += (1 - b1) * gf", "m += b1 * gf"),
    "lower_triangle_order": ("iu = np.triu_indices(9, 1)", "iu = np.tril_indices(9, -1)"),
    "column_major_triangle": ("iu = np.triu_indices(9, 1)",
                              "iu = tuple(a[np.lexsort(np.triu_indices(9, 1))] for a in np.triu_indices(9, 1))"),
    "uncentred_log_scales": ("F[c, 36:45] = ld - ld.mean()", "F[c, 36:45] = ld"),
    "degree_without_log1p": ("np.log1p(degree[c])", "np.log(degree[c] + 2.0)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    mod = _mutant(*MUTANTS[name])
    failed = [p.__name__ for p in PINS if not p(mod)]
    assert failed, f"mutant {name} passes every pin"
