"""The FP32H run expansion's coefficients (``expand`` in ``csrc/gram_exact.hip``) against the
Gegenbauer generating functions they come from (exact near-field distance, Sec. II).

Along a run, an element at offset t from the run centre is at distance
    r(t) = r_c sqrt(1 - 2 mu h + h^2),   h = t / r_c,   mu = (user - centre) . axis / r_c,
so   r(t) = r_c sum_k C_k^(-1/2)(mu) h^k   and   r(t)^-p = r_c^-p sum_k C_k^(p/2)(mu) h^k
(p = 1 free space, p = 3/2 projected aperture).  With t = m' d and q = d / r_c the kernel
carries minus the phase, th[k] = -C_k^(-1/2)(mu) d q^(k-1), and the amplitude,
am[k] = b0 C_k^(p/2)(mu) q^k, each written as products of shared factors and short polynomials
in mu^2.  The second tier's high terms move the phase by about 1e-8 turns and the amplitude by
1e-7 relative, too little for the GPU parity tests to see a wrong constant or factor.

Here the body of ``expand`` is translated statement by statement into Python (its FP32
intrinsics become exact FP64 arithmetic), run for both amplitude models and both tiers, and
every coefficient is held to the Gegenbauer three-term recurrence, to FP64 rounding; the
recurrence itself is held to a direct power series of the generating function."""
import math
import os
import re

import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2503_18118_amd", "csrc", "gram_exact.hip")
AMP_FREESPACE, AMP_PNUSW = 0, 1


def gegenbauer(k, lam, x):
    """C_k^(lam)(x) by the three-term recurrence."""
    c0, c1 = 1.0, 2.0 * lam * x
    if k == 0:
        return c0
    for n in range(2, k + 1):
        c0, c1 = c1, (2.0 * x * (n + lam - 1.0) * c1 - (n + 2.0 * lam - 2.0) * c0) / n
    return c1


def _expand_body():
    src = open(SRC).read()
    start = src.index("Expansion<AMP, TIER> expand(")
    body = src[src.index("{", start) + 1:]
    depth, end = 1, 0
    for i, c in enumerate(body):
        depth += (c == "{") - (c == "}")
        if depth == 0:
            end = i
            break
    body = re.sub(r"//[^\n]*", "", body[:end])
    return body


def _tokens(body):
    """Split into 'if (cond)', 'else', '{', '}' and statements ending in ';'."""
    out, i = [], 0
    while i < len(body):
        if body[i].isspace():
            i += 1
        elif body[i] in "{}":
            out.append(body[i])
            i += 1
        elif body.startswith("if constexpr", i):
            j = body.index("(", i)
            depth = 0
            for k in range(j, len(body)):
                depth += (body[k] == "(") - (body[k] == ")")
                if depth == 0:
                    break
            out.append(("if", body[j + 1:k]))
            i = k + 1
        elif body.startswith("else", i):
            out.append("else")
            i += 4
        else:
            j = body.index(";", i)
            out.append(("stmt", " ".join(body[i:j].split())))
            i = j + 1
    return out


def _py_expr(e):
    e = re.sub(r"(\d+\.\d*)f\b", r"\1", e)
    e = re.sub(r"\((double|float)\)", "", e)
    e = e.replace("__builtin_fmaf", "fma").replace("__builtin_amdgcn_", "")
    e = e.replace("x.th", "th").replace("x.am", "am")
    return e


def _translate(tokens):
    lines, ind, pending = [], 0, False   # pending: an 'if'/'else' without braces covers one statement
    for t in tokens:
        if t == "{":
            pending = False
            continue
        if t == "}":
            ind -= 1
            continue
        if t == "else":
            lines.append("    " * ind + "else:")
            ind += 1
            pending = True
            continue
        kind, text = t
        if kind == "if":
            lines.append("    " * ind + f"if {text}:")
            ind += 1
            pending = True
            continue
        if text.startswith("Expansion<") or text.startswith("return"):
            stmt = None
        else:
            stmt = re.sub(r"^(const\s+)?(double|float)\s+", "", text)
        if stmt is not None:
            lines.append("    " * ind + _py_expr(stmt))
        if pending:
            ind -= 1
            pending = False
    return "\n".join(lines)


PROGRAM = _translate(_tokens(_expand_body()))


def run_expand(amp, tier, dyc, xp2, ds, us):
    env = dict(
        AMP=amp, TIER=tier, XLMIMO_AMP_FREESPACE=AMP_FREESPACE, XLMIMO_AMP_PNUSW=AMP_PNUSW,
        dyc=dyc, xp2=xp2, ds=ds, us=us, th=[None] * 7, am=[None] * 5,
        fma=lambda a, b, c: a * b + c, rsqf=lambda v: 1.0 / math.sqrt(v),
        sqrtf=math.sqrt, fract=lambda v: v - math.floor(v))
    exec(compile(PROGRAM, SRC + ":expand", "exec"), env)
    return env["th"], env["am"]


def test_translation_covers_every_coefficient():
    for amp in (AMP_FREESPACE, AMP_PNUSW):
        th, am = run_expand(amp, 1, 3.0, 500.0 ** 2, 0.5, 1.0)
        assert all(v is not None for v in th[:5]) and th[5] is None
        assert all(v is not None for v in am[:4]) and am[4] is None
        th, am = run_expand(amp, 2, 3.0, 500.0 ** 2, 0.5, 1.0)
        assert all(v is not None for v in th) and all(v is not None for v in am)


CASES = [(dy, x, ds) for dy in (-420.0, -60.0, 0.0, 35.0, 380.0) for x, ds in ((250.0, 0.5), (700.0, 1.0), (95.0, 0.25))]


@pytest.mark.parametrize("amp,lam,p", [(AMP_FREESPACE, 0.5, 1.0), (AMP_PNUSW, 0.75, 1.5)])
@pytest.mark.parametrize("tier,kth,kam", [(1, 4, 3), (2, 6, 4)])
def test_coefficients_follow_the_gegenbauer_series(amp, lam, p, tier, kth, kam):
    us = 0.8   # the per-user scale folded into b0
    for dyc, xp, ds in CASES:
        th, am = run_expand(amp, tier, dyc, xp * xp, ds, us)
        rc = math.hypot(dyc, xp)
        mu, q = dyc / rc, ds / rc
        assert th[0] == pytest.approx(-(rc - math.floor(rc)), abs=1e-12)
        for k in range(1, kth + 1):
            want = -gegenbauer(k, -0.5, mu) * ds * q ** (k - 1)
            assert th[k] == pytest.approx(want, rel=1e-11, abs=1e-15 * ds * q ** (k - 1)), (k, dyc, xp)
        b0 = us * rc ** -p
        for k in range(0, kam + 1):
            want = b0 * gegenbauer(k, lam, mu) * q ** k
            assert am[k] == pytest.approx(want, rel=1e-11, abs=1e-15 * b0 * q ** k), (k, dyc, xp)


def test_a_planted_mistake_is_seen():
    # the same check on a copy of the translation with one tier-2 constant changed in its last digit
    global PROGRAM
    saved = PROGRAM
    PROGRAM = saved.replace("9.0234375", "9.0234376")
    try:
        th, am = run_expand(AMP_PNUSW, 2, 200.0, 300.0 ** 2, 0.5, 1.0)
        rc = math.hypot(200.0, 300.0)
        want = rc ** -1.5 * gegenbauer(4, 0.75, 200.0 / rc) * (0.5 / rc) ** 4
        assert am[4] != pytest.approx(want, rel=1e-11, abs=0.0)
    finally:
        PROGRAM = saved


def test_recurrence_against_the_generating_function():
    # the recurrence, against a direct power series of (1 - 2 mu h + h^2)^(-lam) at small h
    for lam in (-0.5, 0.5, 0.75):
        for mu in (-0.7, 0.0, 0.3, 0.9):
            h = 1e-2
            series = sum(gegenbauer(k, lam, mu) * h ** k for k in range(30))
            assert series == pytest.approx((1.0 - 2.0 * mu * h + h * h) ** (-lam), rel=1e-14)
    # closed forms at low order: C_2^(-1/2) = (1 - mu^2) / 2, P_2 = (3 mu^2 - 1) / 2
    for mu in (-0.4, 0.6):
        assert gegenbauer(2, -0.5, mu) == pytest.approx((1.0 - mu * mu) / 2.0, rel=1e-15)
        assert gegenbauer(2, 0.5, mu) == pytest.approx((3.0 * mu * mu - 1.0) / 2.0, rel=1e-15)
