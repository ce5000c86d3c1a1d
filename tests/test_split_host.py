"""The library's equation reader and split (host code, no GPU) against the
oracle's split of the same text (Sec. 2.4.2): the symbol L(k^2) of every
field, the derivative of its explicit terms and their monomials."""
import os

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
])
def test_library_rejects(L, text, code):
    with pytest.raises(ss.SpecStepError) as e:
        ss.ss_split_equations(text, {})
    assert e.value.code == code


def test_library_rejects_bad_coefficients(L):
    for coefs in ({"psi": 1.0}, {"lap": 1.0}, {"a": float("nan")}, {"1a": 1.0}):
        with pytest.raises(ss.SpecStepError) as e:
            ss.ss_split_equations("psi' = -psi", coefs)
        assert e.value.code == 1
