"""The matrix-core screen's error model, probed on the hardware: every sum
A X + B Y + c that v_mfma_f32_32x32x2f32 forms (the margin of Eq. 11 in the
matrix-core screen) lies within 4 u of the sum of |A X|, |B Y| and |c| from
the exact value (u = 2^-24; the screen's band assumes this, 6.05 u in all
with the coefficient and coordinate roundings), on adversarial operands:
near-complete cancellation, mixed magnitudes over 2^-60..2^60, products in
and below the float32 subnormal range (an absolute 2^-126 allowance, far
below the band's absolute term), signed zeros and exact ties."""
from __future__ import annotations

import sys
from fractions import Fraction as Fr

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U = 2.0 ** -24


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_15385_amd as P
    P.load_library()
    return P


def f32(x):
    return np.asarray(x, dtype=np.float32)


def adversarial(rng, k):
    """k entries (A, B, c, X, Y) of each kind."""
    out = []
    mag = lambda lo, hi, n: (2.0 ** rng.uniform(lo, hi, n)) * rng.choice([-1.0, 1.0], n)
    # 1. random magnitudes
    out.append(np.stack([mag(-60, 60, k), mag(-60, 60, k), mag(-60, 60, k), mag(-30, 30, k),
                         mag(-30, 30, k)], 1))
    # 2. A X + B Y ~ 0 (B chosen so that B Y cancels A X), c small or zero
    A, X, Y = mag(-10, 10, k), mag(-10, 10, k), mag(-10, 10, k)
    B = -f32(A * X / Y).astype(np.float64)
    out.append(np.stack([A, B, mag(-40, -20, k) * (rng.random(k) < 0.5), X, Y], 1))
    # 3. c cancels A X + B Y (rounded), leaving the rounding residue
    A, B, X, Y = mag(-5, 5, k), mag(-5, 5, k), mag(-5, 5, k), mag(-5, 5, k)
    c = -f32(A.astype(np.float32).astype(np.float64) * X + B * Y).astype(np.float64)
    out.append(np.stack([A, B, c, X, Y], 1))
    # 4. mixed magnitudes: one huge term cancelled by c, one small term
    A, X = mag(15, 20, k), mag(15, 20, k)
    c = -f32(A * X).astype(np.float64)
    out.append(np.stack([A, mag(-3, 3, k), c, X, mag(-3, 3, k)], 1))
    # 5. products near and below the subnormal range
    out.append(np.stack([mag(-75, -55, k), mag(-75, -55, k), mag(-150, -110, k) * (rng.random(k) < 0.5),
                         mag(-75, -55, k), mag(-75, -55, k)], 1))
    # 6. signed zeros and exact small integers (exact sums)
    z = rng.choice([0.0, -0.0, 1.0, -1.0, 2.0, 3.0], size=(k, 5))
    out.append(z)
    return f32(np.concatenate(out))


def exact_sum(e):
    A, B, c, X, Y = (Fr(float(v)) for v in e)
    terms = (A * X, B * Y, c)
    return sum(terms), sum(abs(t) for t in terms)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mfma_sum_within_model(P, seed):
    rng = np.random.default_rng(900 + seed)
    ent = adversarial(rng, 3000)
    got = P.pip_mfma_margin_probe(torch.from_numpy(ent).cuda()).cpu().numpy()
    worst = 0.0
    bad = []
    for i, e in enumerate(ent):
        ex, mag = exact_sum(e)
        err = abs(Fr(float(got[i])) - ex)
        allow = 4 * Fr(U) * mag + 4 * Fr(2.0 ** -126)
        if mag > 0:
            worst = max(worst, float(err / (Fr(U) * mag)))
        if err > allow:
            bad.append((i, e.tolist(), float(got[i]), float(ex)))
    say(f"[stat] matrix-core sum: worst error {worst:.3f} u of the sum of |terms| "
        f"over {len(ent)} adversarial entries")
    assert not bad, bad[:5]
