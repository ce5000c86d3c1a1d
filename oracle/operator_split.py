"""Generic operator split of an equation of motion, plain FP64 (oracle).

TEST INFRASTRUCTURE ONLY: used by tests; never by the product path.

What is computed (Sec. 2.4.2, the procedure that turns any equation of
motion into the spectral scheme, and its update rule):
  * the right-hand side of each field's equation is expanded into terms
    c * lap^p (m), m a monomial in the fields;
  * step 1: the terms split into the linear part (degree <= 1 in the
    fields, constants included) and the nonlinear part N (degree >= 2);
  * step 2: the linear part splits again into L_psi, the terms linear in
    the field itself, and L_*, the rest (constants, other fields);
  * step 3: L_psi with the field removed and lap -> -|k|^2 is the symbol
    L(k), which gives A;
  * steps 4-6: L_* and N are each written as a sum of distinct
    derivatives d applied to expressions e: the sets D_* and D_N;
  * step 7: elements of D_* and D_N with the same derivative are paired,
    an element with no partner is paired with 0 (D = D_1 u D_2 u D_3);
  * step 8: B_i = B d_i(k) and E_i = (e from D_*, e from D_N);
  * the step: psi_hat' = A psi_hat + sum_i B_i FFT(E_i^0 + E_i^1).

Two choices of (A, B) from L(k):
  * "etd1": A = exp(L dt), B = (exp(L dt) - 1)/L (Eq. 4; B = dt at L = 0),
    the scheme the paper prints;
  * "implicit": A = 1/(1 - L dt), B = dt/(1 - L dt), the linearly
    implicit first-order scheme of the semi-implicit family the paper
    cites (same first-order accuracy; needs 1 - L dt > 0 at every mode).

Readings taken where the paper is silent:
  * "linear" counts constant terms and terms in the other fields: they
    are the L_* of step 2, handled as explicit terms with N;
  * a derivative multiplied by a field (psi lap psi) cannot be written
    as an operator applied to a pointwise function: it is rejected;
  * derivatives are powers of the Laplacian only (lap, bilap), with the
    continuous symbol lap -> -|k|^2, k_j = 2 pi m_j / (N_j dx_j);
  * all fields on the right-hand side are taken at the current step.

Equation text: one equation per field, separated by ';' or newlines,
each "name' = expression".  Expressions use numbers, coefficient names,
field names, + - * /, '^' (or '**') with a non-negative integer literal
exponent, parentheses, lap(...) and bilap(...) (= lap(lap(...))).
Division is by constant expressions only.
"""
from __future__ import annotations

import re

import numpy as np


class SplitError(ValueError):
    """The text is not an equation this split can represent."""


_TOKEN = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][+-]?\d+)?|\.\d+(?:[eE][+-]?\d+)?|\d+(?:[eE][+-]?\d+)?)"
                    r"|([A-Za-z_][A-Za-z_0-9]*)|(\*\*|[-+*/^()']|=))")


def _tokens(text):
    out, pos = [], 0
    text = text.rstrip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            raise SplitError("cannot read %r" % text[pos:pos + 10])
        num, name, op = m.groups()
        out.append(("num", float(num)) if num else ("name", name) if name else ("op", op))
        pos = m.end()
    return out


class _Expr:
    """A sum of terms {(p, exps): c}: c * lap^p applied to prod f_j^exps_j."""

    def __init__(self, nf, terms=None):
        self.nf = nf
        self.terms = {}
        for k, c in (terms or {}).items():
            self._add(k, c)

    def _add(self, key, c):
        v = self.terms.get(key, 0.0) + c
        if v == 0.0:
            self.terms.pop(key, None)
        else:
            self.terms[key] = v

    @classmethod
    def const(cls, nf, v):
        return cls(nf, {(0, (0,) * nf): float(v)})

    @classmethod
    def field(cls, nf, j):
        e = [0] * nf
        e[j] = 1
        return cls(nf, {(0, tuple(e)): 1.0})

    def is_const(self):
        return all(p == 0 and not any(e) for p, e in self.terms)

    def const_value(self):
        return self.terms.get((0, (0,) * self.nf), 0.0)

    def plus(self, other, sign=1.0):
        r = _Expr(self.nf, self.terms)
        for k, c in other.terms.items():
            r._add(k, sign * c)
        return r

    def times(self, other):
        r = _Expr(self.nf)
        for (pa, ea), ca in self.terms.items():
            for (pb, eb), cb in other.terms.items():
                if (pa > 0 and any(eb)) or (pb > 0 and any(ea)):
                    raise SplitError("a derivative multiplied by a field has no operator form")
                r._add((pa + pb, tuple(x + y for x, y in zip(ea, eb))), ca * cb)
        return r

    def lap(self, times=1):
        r = _Expr(self.nf)
        for (p, e), c in self.terms.items():
            if any(e):                      # the Laplacian of a constant is zero
                r._add((p + times, e), c)
        return r


class _Parser:
    def __init__(self, toks, fields, coefs):
        self.t, self.i = toks, 0
        self.fields, self.coefs = fields, coefs
        self.nf = len(fields)

    def peek(self):
        return self.t[self.i] if self.i < len(self.t) else (None, None)

    def take(self, kind=None, val=None):
        tok = self.peek()
        if tok[0] is None or (kind and tok[0] != kind) or (val is not None and tok[1] != val):
            raise SplitError("expected %s, found %r" % (val or kind, tok[1]))
        self.i += 1
        return tok

    def expr(self):
        r = self.product()
        while self.peek() in (("op", "+"), ("op", "-")):
            sign = 1.0 if self.take()[1] == "+" else -1.0
            r = r.plus(self.product(), sign)
        return r

    def product(self):
        r = self.unary()
        while self.peek() in (("op", "*"), ("op", "/")):
            op = self.take()[1]
            rhs = self.unary()
            if op == "*":
                r = r.times(rhs)
            else:
                if not rhs.is_const() or rhs.const_value() == 0.0:
                    raise SplitError("division by a non-constant or zero expression")
                r = r.times(_Expr.const(self.nf, 1.0 / rhs.const_value()))
        return r

    def unary(self):
        if self.peek() == ("op", "-"):
            self.take()
            return _Expr.const(self.nf, -1.0).times(self.unary())
        if self.peek() == ("op", "+"):
            self.take()
            return self.unary()
        return self.power()

    def power(self):
        base = self.atom()
        if self.peek() in (("op", "^"), ("op", "**")):
            self.take()
            kind, v = self.take("num")
            if v != int(v) or v < 0:
                raise SplitError("exponents are non-negative integers")
            r = _Expr.const(self.nf, 1.0)
            for _ in range(int(v)):
                r = r.times(base)
            if self.peek() in (("op", "^"), ("op", "**")):
                raise SplitError("chained exponents are ambiguous; use parentheses")
            return r
        return base

    def atom(self):
        kind, v = self.take()
        if kind == "num":
            return _Expr.const(self.nf, v)
        if kind == "name":
            if v in ("lap", "bilap"):
                self.take("op", "(")
                inner = self.expr()
                self.take("op", ")")
                return inner.lap(1 if v == "lap" else 2)
            if v in self.fields:
                return _Expr.field(self.nf, self.fields.index(v))
            if v in self.coefs:
                return _Expr.const(self.nf, self.coefs[v])
            raise SplitError("unknown name %r" % v)
        if v == "(":
            r = self.expr()
            self.take("op", ")")
            return r
        raise SplitError("unexpected %r" % v)


class Split:
    """Result of the procedure for every field j:
    ``L[j]``        {p: c}, the symbol L(k) = sum_p c (-|k|^2)^p;
    ``channels[j]`` list of (p, E0, E1): derivative lap^p applied to
                    E0 (from L_*) + E1 (from N), each {exps: c}."""

    def __init__(self, fields, L, channels):
        self.fields, self.L, self.channels = fields, L, channels


def parse(text, coefs=None):
    """Equation text -> Split (steps 1-8 of the procedure)."""
    coefs = dict(coefs or {})
    eqs = [s for s in re.split(r"[;\n]", text) if s.strip()]
    lhs, rhs = [], []
    for s in eqs:
        toks = _tokens(s)
        if len(toks) < 4 or toks[0][0] != "name" or toks[1] != ("op", "'") or toks[2] != ("op", "="):
            raise SplitError("each equation reads  name' = expression")
        lhs.append(toks[0][1])
        rhs.append(toks[3:])
    if len(set(lhs)) != len(lhs):
        raise SplitError("a field has two equations")
    for name in lhs:
        if name in coefs or name in ("lap", "bilap"):
            raise SplitError("%r is both a field and another name" % name)
    L, channels = [], []
    for j, toks in enumerate(rhs):
        p = _Parser(toks, lhs, coefs)
        e = p.expr()
        if p.i != len(toks):
            raise SplitError("trailing text in the equation of %r" % lhs[j])
        unit = tuple(1 if f == j else 0 for f in range(len(lhs)))
        # step 1: linear (degree <= 1) and nonlinear parts
        linear = {k: c for k, c in e.terms.items() if sum(k[1]) <= 1}
        nonlin = {k: c for k, c in e.terms.items() if sum(k[1]) >= 2}
        # steps 2-3: L_psi (the field itself, removed) and L_*
        Lpsi = {pw: c for (pw, ex), c in linear.items() if ex == unit}
        Lstar = {(pw, ex): c for (pw, ex), c in linear.items() if ex != unit}
        # steps 4-6: unique derivatives applied to expressions
        def by_derivative(terms):
            d = {}
            for (pw, ex), c in terms.items():
                d.setdefault(pw, {})[ex] = c
            return d
        Dstar, DN = by_derivative(Lstar), by_derivative(nonlin)
        # step 7: pair on equal derivatives, 0 where one side has none
        chans = [(pw, Dstar.get(pw, {}), DN.get(pw, {})) for pw in sorted(set(Dstar) | set(DN))]
        L.append(Lpsi)
        channels.append(chans)
    return Split(lhs, L, channels)


def wavenumber_sq(shape, dx):
    """|k|^2 on the FFT grid of an array shaped (..., y, x); dx in (x, y[, z])."""
    dxs = tuple(reversed(tuple(dx)))
    k2 = np.zeros(tuple(shape))
    for ax, (n, h) in enumerate(zip(shape, dxs)):
        k = 2.0 * np.pi * np.fft.fftfreq(n, d=h)
        sl = [None] * len(shape)
        sl[ax] = slice(None)
        k2 = k2 + (k ** 2)[tuple(sl)]
    return k2


def symbol(poly, k2):
    """sum_p c (-|k|^2)^p: lap -> -|k|^2 (step 3)."""
    out = np.zeros_like(k2)
    for p, c in poly.items():
        out = out + c * (-k2) ** p
    return out


def factors(L, dt, scheme):
    """(A, B) of one field from its symbol L(k)."""
    z = L * dt
    if scheme == "etd1":
        phi = np.ones_like(z)
        nz = z != 0.0
        phi[nz] = np.expm1(z[nz]) / z[nz]
        return np.exp(z), dt * phi
    if scheme == "implicit":
        den = 1.0 - z
        if np.any(den <= 0.0):
            raise SplitError("1 - L dt is not positive at every mode")
        return 1.0 / den, dt / den
    raise SplitError("unknown scheme %r" % scheme)


def pointwise(expr, q):
    """sum c prod_f q_f^e_f at every cell."""
    out = np.zeros_like(q[0])
    for ex, c in expr.items():
        t = np.full_like(q[0], c)
        for f, n in enumerate(ex):
            for _ in range(n):
                t = t * q[f]
        out = out + t
    return out


def step_n(fields, split, dt, dx, nsteps, scheme="etd1"):
    """``nsteps`` steps of psi_hat' = A psi_hat + sum_i B_i FFT(E_i^0 + E_i^1)."""
    q = [np.array(f, dtype=np.float64, copy=True) for f in fields]
    if len(q) != len(split.fields):
        raise SplitError("%d fields given, the equations have %d" % (len(q), len(split.fields)))
    k2 = wavenumber_sq(q[0].shape, dx)
    tables = []
    for j in range(len(q)):
        A, B = factors(symbol(split.L[j], k2), dt, scheme)
        Bi = [(B * symbol({p: 1.0}, k2), e0, e1) for p, e0, e1 in split.channels[j]]
        tables.append((A, Bi))
    for _ in range(int(nsteps)):
        new = []
        for j, (A, Bi) in enumerate(tables):
            acc = A * np.fft.fftn(q[j])
            for b, e0, e1 in Bi:
                acc = acc + b * np.fft.fftn(pointwise(e0, q) + pointwise(e1, q))
            new.append(np.ascontiguousarray(np.fft.ifftn(acc).real))
        q = new
    return q


def euler_n(fields, split, dt, dx, nsteps, stencil=0):
    """``nsteps`` forward-Euler steps (Sec. 2.4.1) of the split equations
    with finite-difference Laplacians (Sec. 2.2.2, the stencils of
    ``fd_euler.laplacian``): psi_j' = psi_j + dt (sum_p c_p lap^p psi_j +
    sum_i lap^p_i (E_i^0 + E_i^1)), every term from the fields of the
    current step."""
    from oracle.fd_euler import laplacian

    def lap_pow(f, p):
        for _ in range(p):
            f = laplacian(f, dx, stencil)
        return f

    q = [np.array(f, dtype=np.float64, copy=True) for f in fields]
    if len(q) != len(split.fields):
        raise SplitError("%d fields given, the equations have %d" % (len(q), len(split.fields)))
    for _ in range(int(nsteps)):
        new = []
        for j in range(len(q)):
            rhs = np.zeros_like(q[j])
            for p, c in split.L[j].items():
                rhs = rhs + c * lap_pow(q[j], p)
            for p, e0, e1 in split.channels[j]:
                rhs = rhs + lap_pow(pointwise(e0, q) + pointwise(e1, q), p)
            new.append(q[j] + dt * rhs)
        q = new
    return q
