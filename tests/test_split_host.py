"""The library's equation reader and split (host code, no GPU) against the
oracle's split of the same text (Sec. 2.4.2): the symbol L(k^2) of every
field, the derivative of its explicit terms and their monomials."""
import os

import numpy as np
import pytest

from oracle import operator_split as osp
from paper_2109_02598_amd import specstep as ss
from tests import _equations as eqs
from tests._common import COEF


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ss.LIB_PATH):
        pytest.skip("library not built")
    return ss.lib()


def oracle_tables(text, coefs):
    """The oracle's split in the library's layout: L as coefficients of
    k^(2p) ((-1)^p c) and each explicit channel (ascending p) as one
    monomial map of its paired L_* and N terms."""
    sp = osp.parse(text, coefs)
    out = []
    for j in range(len(sp.fields)):
        Lc = [0.0] * 4
        for p, c in sp.L[j].items():
            Lc[p] += c * (-1) ** p
        chans = []
        for pw, e0, e1 in sp.channels[j]:
            terms = {}
            for ex, c in list(e0.items()) + list(e1.items()):
                key = tuple(ex) + (0,) * (2 - len(ex))
                terms[key] = terms.get(key, 0.0) + c
            chans.append((pw, terms))
        out.append((Lc, chans))
    return out


TEXTS = [eqs.fixed(m, COEF[m]) for m in ("allen_cahn", "cahn_hilliard", "gray_scott", "model_c")] + [
    eqs.fixed("pfc", (-0.25, 1.0, 0.3, 1.0)),
    eqs.fixed("cahn_hilliard", (1.7, 0.6, -0.4, 2.5)),
    eqs.SWIFT_HOHENBERG, eqs.FITZHUGH_NAGUMO, eqs.CONSERVED_QUARTIC,
    ("a' = -a + lap(b + 0.2*b^2); b' = 0.5*lap(b) - a*b + 0.05 - 3", {}),   # L_* and N paired under lap
    ("x' = (x + 2)^3 - x^3 - 6*x^2 - 0.5*(x - 1)*(x + 1)", {}),       # cancellations
    ("x' = lap(x)*3/4 + 1e-3*bilap(x) - lap(lap(lap(x))) + x**2/3", {}),
    ("p' = -(p - q)^2 + lap(2*p); q' = q - p*q", {}),
    # two explicit channels per field (identity and a Laplacian power)
    ("psi' = lap(psi) - psi^3 + 0.5*lap(psi^3)", {}),
    ("u' = 0.2*lap(u) - u*v^2 + 0.03*(1 - u) + 0.01*lap(u^2*v); v' = 0.1*lap(v) + u*v^2 - 0.09*v", {}),
    ("phi' = lap(phi^3 - phi - lap(phi)) + 0.02*bilap(phi^2)", {}),
    ("a' = -a + lap(b + 0.2*b^2) + a*b; b' = 0.5*lap(b) - a*b + 0.05 - bilap(a^2)*0.01", {}),
]


@pytest.mark.parametrize("case", range(len(TEXTS)))
def test_library_split_matches_the_oracle(L, case):
    text, coefs = TEXTS[case]
    got = ss.ss_split_equations(text, coefs)
    want = oracle_tables(text, coefs)
    assert len(got) == len(want)
    for g, (Lc, chans) in zip(got, want):
        assert g["L"] == pytest.approx(Lc, rel=1e-14, abs=1e-15)
        assert [c["p"] for c in g["channels"]] == [p for p, _ in chans]
        for gc, (p, terms) in zip(g["channels"], chans):
            gt = {(e0, e1): c for c, e0, e1 in gc["terms"]}
            # exact zeros are dropped by both; tiny residues of cancellation may not be
            keys = {k for k in set(gt) | set(terms) if abs(gt.get(k, 0.0)) > 1e-14 or abs(terms.get(k, 0.0)) > 1e-14}
            for k in keys:
                assert gt.get(k, 0.0) == pytest.approx(terms.get(k, 0.0), rel=1e-14, abs=1e-14), (p, k)


@pytest.mark.parametrize("text,code", [
    ("psi' = psi*lap(psi)", 2), ("psi' = psi/psi", 2), ("psi' = psi^2.5", 2), ("psi' = foo", 1),
    ("psi' = 2 psi", 1), ("psi' = psi^2^2", 1), ("psi = psi", 1), ("psi' = lap psi", 1),
    ("psi' = psi; psi' = -psi", 1), ("psi' = (psi", 1), ("", 1),
    ("psi' = lap(psi) - psi^3 + lap(psi^2) + bilap(psi^2)", 2),   # three derivatives: two per field
    ("psi' = bilap(bilap(psi^3))", 2),               # explicit terms under lap^4 (lap^3 is the highest)
    ("psi' = lap(lap(bilap(psi)))", 2),              # L above lap^3
    ("a' = a; b' = b; c' = c", 2),                   # three fields
    ("psi' = psi^8", 2),                             # exponent above 7
    ("psi' = (1 + psi)^9 - psi^9", 2),               # more than 8 monomials
    ("psi' = " + "(" * 201 + "psi" + ")" * 201, 1),  # nesting beyond the bound
    ("psi' = " + "-" * 201 + "psi", 1),
    ("psi' = " + "lap(" * 201 + "psi" + ")" * 201, 1),
])
def test_library_rejects(L, text, code):
    with pytest.raises(ss.SpecStepError) as e:
        ss.ss_split_equations(text, {})
    assert e.value.code == code


def test_library_survives_deep_nesting(L):
    """Nesting far past the bound is refused, not a stack overflow; at the
    bound it is read."""
    for n in (10 ** 5, 10 ** 6):
        for text in ("psi' = " + "(" * n + "psi" + ")" * n, "psi' = " + "-" * n + "psi",
                     "psi' = " + "+" * n + "psi", "psi' = " + "lap(" * n + "psi" + ")" * n):
            with pytest.raises(ss.SpecStepError) as e:
                ss.ss_split_equations(text, {})
            assert e.value.code == 1
    got = ss.ss_split_equations("psi' = " + "(" * 199 + "-psi" + ")" * 199, {})
    assert got[0]["L"] == pytest.approx([-1.0, 0.0, 0.0, 0.0])


def test_library_rejects_bad_coefficients(L):
    for coefs in ({"psi": 1.0}, {"lap": 1.0}, {"a": float("nan")}, {"1a": 1.0}):
        with pytest.raises(ss.SpecStepError) as e:
            ss.ss_split_equations("psi' = -psi", coefs)
        assert e.value.code == 1


TOKENS = ["psi", "u", "v", "lap(", "bilap(", "(", ")", "+", "-", "*", "/", "^", "**", "2", "3", "0.5",
          "1e3", "7", "16", "'", "=", ";", " ", "\n", "c", "psi'", "u'", "v'", "=", ".", "e", "1e309"]


def test_reader_never_crashes_on_token_soup(L):
    """Seeded random token strings (and prefixes of valid equations):
    every one is read or refused with an error code, never a crash."""
    rng = np.random.default_rng(2109)
    texts = []
    for _ in range(3000):
        k = int(rng.integers(1, 40))
        texts.append("".join(TOKENS[i] for i in rng.integers(0, len(TOKENS), k)))
    for text, _ in TEXTS:
        texts += [text[:i] for i in range(len(text) + 1)]
    ok = 0
    for t in texts:
        try:
            ss.ss_split_equations(t, {"c": 0.5})
            ok += 1
        except ss.SpecStepError as e:
            assert e.code in (1, 2), (t, e.code)
    assert ok > 0


def random_equations(rng, count):
    """Seeded random equations of the reader's grammar (one or two fields,
    the coefficient c, nested sums, products, small powers, lap/bilap).  A
    derivative is multiplied by a constant only, as the split requires."""
    def atom(fields, depth):
        r = rng.random()
        if depth > 2 or r < 0.45:
            return str(fields[int(rng.integers(len(fields)))])
        if r < 0.65:
            return "%g" % round(float(rng.uniform(-2, 2)), 3)
        if r < 0.75:
            return "c"
        return "(" + expr(fields, depth + 1, False) + ")"

    def term(fields, depth, deriv):
        if deriv and depth < 3 and rng.random() < 0.35:
            op = "lap" if rng.random() < 0.8 else "bilap"
            return "%g*%s(%s)" % (round(float(rng.uniform(-2, 2)), 3), op, expr(fields, depth + 1, True))
        t = atom(fields, depth)
        if rng.random() < 0.25:
            t += "^%d" % int(rng.integers(0, 4))
        for _ in range(int(rng.integers(0, 3))):
            t += "*" + atom(fields, depth) if rng.random() < 0.85 else "/%g" % float(rng.choice([2, 4, 0.5]))
        return t

    def expr(fields, depth, deriv=True):
        e = ("-" if rng.random() < 0.2 else "") + term(fields, depth, deriv)
        for _ in range(int(rng.integers(0, 4))):
            e += (" + " if rng.random() < 0.5 else " - ") + term(fields, depth, deriv)
        return e

    out = []
    for _ in range(count):
        fields = ["psi"] if rng.random() < 0.6 else ["u", "v"]
        out.append("; ".join("%s' = %s" % (f, expr(fields, 0)) for f in fields))
    return out


def test_random_equations_split_like_the_oracle(L):
    """Differential check on seeded random equations: whenever the library
    takes a text, the oracle's split of it gives the same tables; a text
    the library cannot read is one the oracle cannot read either."""
    rng = np.random.default_rng(2109)
    taken = refused = 0
    for text in random_equations(rng, 400):
        coefs = {"c": 0.75}
        try:
            got = ss.ss_split_equations(text, coefs)
        except ss.SpecStepError as e:
            refused += 1
            if e.code == 1:
                with pytest.raises(Exception):
                    osp.parse(text, coefs)
            continue
        taken += 1
        want = oracle_tables(text, coefs)
        assert len(got) == len(want), text
        for g, (Lc, chans) in zip(got, want):
            assert g["L"] == pytest.approx(Lc, rel=1e-12, abs=1e-12), text
            assert [c["p"] for c in g["channels"]] == [p for p, _ in chans], text
            for gc, (p, terms) in zip(g["channels"], chans):
                gt = {(e0, e1): c for c, e0, e1 in gc["terms"]}
                keys = {k for k in set(gt) | set(terms)
                        if abs(gt.get(k, 0.0)) > 1e-12 or abs(terms.get(k, 0.0)) > 1e-12}
                for k in keys:
                    assert gt.get(k, 0.0) == pytest.approx(terms.get(k, 0.0), rel=1e-12, abs=1e-12), (text, p, k)
    assert taken >= 100 and refused >= 20, (taken, refused)
