// Equation text -> spectral-scheme tables (Sec. 2.4.2).
//
// The right-hand side of each field's equation is read into a sum of
// terms c * lap^p (monomial in the fields): products expand, the Laplacian
// distributes over sums and annihilates constants.  A derivative multiplied
// by a field (psi lap psi) has no operator form and is refused.  The split
// then follows the procedure of Sec. 2.4.2:
//   * the terms linear in the field itself form L_psi; with the field
//     removed and lap -> -k^2 they give the symbol L(k^2), hence A;
//   * every other term (constants and terms in other fields, the L_* of
//     the procedure; nonlinear terms, the N) is explicit; explicit terms
//     under the same derivative d are paired into one channel d applied to
//     E, with B d as its operator.
// The GPU step evaluates each channel's E pointwise from a table of
// monomials; a field carries up to two channels, d = lap^p with p <= 3.
//
// Text: one equation per field, separated by ';' or newlines, each
// "name' = expression"; numbers, coefficient names, field names, + - * /,
// '^' or '**' with an integer literal exponent, parentheses, lap(.) and
// bilap(.); division by constants only.

#include "ss_equation.hpp"

#include <cmath>
#include <cctype>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

namespace ss {
namespace {

struct Fail {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  throw Fail{code, buf};
}

// c * lap^p applied to f0^e0 f1^e1
struct Term {
  int p;
  int e[2];
  double c;
};

struct Poly {
  std::vector<Term> t;

  void add(const Term& x) {
    for (Term& y : t)
      if (y.p == x.p && y.e[0] == x.e[0] && y.e[1] == x.e[1]) {
        y.c += x.c;
        return;
      }
    t.push_back(x);
  }
  void prune() {
    std::vector<Term> k;
    for (const Term& x : t)
      if (x.c != 0.0) k.push_back(x);
    t.swap(k);
  }
  // true (and the value) when every term is a plain constant
  bool constant(double* v) const {
    double s = 0;
    for (const Term& x : t) {
      if (x.p != 0 || x.e[0] != 0 || x.e[1] != 0) return false;
      s += x.c;
    }
    *v = s;
    return true;
  }
  static Poly num(double v) {
    Poly r;
    r.t.push_back(Term{0, {0, 0}, v});
    r.prune();
    return r;
  }
};

Poly mul(const Poly& a, const Poly& b) {
  Poly r;
  for (const Term& x : a.t)
    for (const Term& y : b.t) {
      const bool xf = x.e[0] || x.e[1], yf = y.e[0] || y.e[1];
      if ((x.p > 0 && yf) || (y.p > 0 && xf))
        fail(2, "a derivative multiplied by a field has no operator form");
      const int e0 = x.e[0] + y.e[0], e1 = x.e[1] + y.e[1];
      if (e0 > 64 || e1 > 64) fail(2, "a monomial's degree is too high");
      r.add(Term{x.p + y.p, {e0, e1}, x.c * y.c});
    }
  r.prune();
  return r;
}

Poly lap(const Poly& a, int times) {
  Poly r;
  for (const Term& x : a.t)
    if (x.e[0] || x.e[1]) r.add(Term{x.p + times, {x.e[0], x.e[1]}, x.c});
  r.prune();
  return r;
}

enum Tok { T_END, T_NUM, T_NAME, T_OP };

class Reader {
 public:
  Reader(const std::string& s, const std::vector<std::string>& fields, const std::vector<std::string>& names,
         const std::vector<double>& values)
      : s_(s), fields_(fields), names_(names), values_(values) {
    next();
  }

  Tok kind() const { return kind_; }
  const std::string& text() const { return tok_; }
  bool at_op(const char* op) const { return kind_ == T_OP && tok_ == op; }

  void expect_op(const char* op) {
    if (!at_op(op)) fail(1, "expected '%s' near '%s'", op, tok_.c_str());
    next();
  }

  std::string take_name() {
    if (kind_ != T_NAME) fail(1, "expected a name near '%s'", tok_.c_str());
    std::string n = tok_;
    next();
    return n;
  }

  Poly sum() {
    Poly r = product();
    while (at_op("+") || at_op("-")) {
      const double sg = at_op("+") ? 1.0 : -1.0;
      next();
      Poly b = product();
      for (Term x : b.t) {
        x.c *= sg;
        r.add(x);
      }
      r.prune();
    }
    return r;
  }

 private:
  Poly product() {
    Poly r = signed_factor();
    while (at_op("*") || at_op("/")) {
      const bool div = at_op("/");
      next();
      Poly b = signed_factor();
      if (div) {
        double v = 0;
        if (!b.constant(&v) || v == 0.0) fail(2, "division by a non-constant or zero expression");
        b = Poly::num(1.0 / v);
      }
      r = mul(r, b);
    }
    return r;
  }

  Poly signed_factor() {
    if (at_op("-")) {
      next();
      Nest nest(*this);
      return mul(Poly::num(-1.0), signed_factor());
    }
    if (at_op("+")) {
      next();
      Nest nest(*this);
      return signed_factor();
    }
    return power();
  }

  Poly power() {
    Poly b = atom();
    if (!(at_op("^") || at_op("**"))) return b;
    next();
    if (kind_ != T_NUM) fail(1, "an exponent must be an integer literal");
    const double v = num_;
    if (v != std::floor(v) || v < 0 || v > 16) fail(2, "exponent %g: integers 0..16 only", v);
    next();
    if (at_op("^") || at_op("**")) fail(1, "chained exponents are ambiguous; use parentheses");
    Poly r = Poly::num(1.0);
    for (int i = 0; i < (int)v; ++i) r = mul(r, b);
    return r;
  }

  Poly atom() {
    if (kind_ == T_NUM) {
      const double v = num_;
      next();
      return Poly::num(v);
    }
    if (kind_ == T_NAME) {
      const std::string n = tok_;
      next();
      if (n == "lap" || n == "bilap") {
        expect_op("(");
        Nest nest(*this);
        Poly in = sum();
        expect_op(")");
        return lap(in, n == "lap" ? 1 : 2);
      }
      for (size_t j = 0; j < fields_.size(); ++j)
        if (fields_[j] == n) {
          Poly r;
          Term x{0, {0, 0}, 1.0};
          x.e[j] = 1;
          r.t.push_back(x);
          return r;
        }
      for (size_t i = 0; i < names_.size(); ++i)
        if (names_[i] == n) return Poly::num(values_[i]);
      fail(1, "unknown name '%s'", n.c_str());
    }
    if (at_op("(")) {
      next();
      Nest nest(*this);
      Poly r = sum();
      expect_op(")");
      return r;
    }
    fail(1, "unexpected '%s'", kind_ == T_END ? "end of equation" : tok_.c_str());
  }

  void next() {
    while (pos_ < s_.size() && std::isspace((unsigned char)s_[pos_])) ++pos_;
    if (pos_ >= s_.size()) {
      kind_ = T_END;
      tok_.clear();
      return;
    }
    const char ch = s_[pos_];
    const size_t b = pos_;
    if (std::isdigit((unsigned char)ch) || ch == '.') {
      // digits [ . digits ] [ e [+-] digits ]
      while (pos_ < s_.size() && std::isdigit((unsigned char)s_[pos_])) ++pos_;
      if (pos_ < s_.size() && s_[pos_] == '.') {
        ++pos_;
        while (pos_ < s_.size() && std::isdigit((unsigned char)s_[pos_])) ++pos_;
      }
      if (pos_ < s_.size() && (s_[pos_] == 'e' || s_[pos_] == 'E')) {
        size_t q = pos_ + 1;
        if (q < s_.size() && (s_[q] == '+' || s_[q] == '-')) ++q;
        if (q < s_.size() && std::isdigit((unsigned char)s_[q])) {
          pos_ = q;
          while (pos_ < s_.size() && std::isdigit((unsigned char)s_[pos_])) ++pos_;
        }
      }
      tok_ = s_.substr(b, pos_ - b);
      if (tok_ == ".") fail(1, "a lone '.'");
      num_ = std::strtod(tok_.c_str(), nullptr);
      if (!std::isfinite(num_)) fail(1, "number '%s' out of range", tok_.c_str());
      kind_ = T_NUM;
      return;
    }
    if (std::isalpha((unsigned char)ch) || ch == '_') {
      while (pos_ < s_.size() && (std::isalnum((unsigned char)s_[pos_]) || s_[pos_] == '_')) ++pos_;
      tok_ = s_.substr(b, pos_ - b);
      kind_ = T_NAME;
      return;
    }
    if (ch == '*' && pos_ + 1 < s_.size() && s_[pos_ + 1] == '*') {
      pos_ += 2;
      tok_ = "**";
      kind_ = T_OP;
      return;
    }
    if (std::strchr("+-*/^()'=", ch)) {
      ++pos_;
      tok_ = std::string(1, ch);
      kind_ = T_OP;
      return;
    }
    fail(1, "unexpected character '%c'", ch);
  }

  // Parentheses, lap(...) and unary signs recurse: their nesting is
  // bounded so that no text can exhaust the caller's stack.
  static constexpr int kMaxDepth = 200;
  struct Nest {
    Reader& r;
    explicit Nest(Reader& rd) : r(rd) {
      if (++r.depth_ > kMaxDepth) fail(1, "expression nested deeper than %d levels", kMaxDepth);
    }
    ~Nest() { --r.depth_; }
  };

  const std::string& s_;
  const std::vector<std::string>& fields_;
  const std::vector<std::string>& names_;
  const std::vector<double>& values_;
  size_t pos_ = 0;
  Tok kind_ = T_END;
  std::string tok_;
  double num_ = 0;
  int depth_ = 0;
};

bool is_ident(const char* s) {
  if (!s || !(std::isalpha((unsigned char)s[0]) || s[0] == '_')) return false;
  for (const char* q = s; *q; ++q)
    if (!(std::isalnum((unsigned char)*q) || *q == '_')) return false;
  return true;
}

void split_all(const char* text, const char* const names[], const double values[], int nvalues, EqSplit* out) {
  if (!text) fail(1, "null equation text");
  if (nvalues < 0 || (nvalues > 0 && (!names || !values))) fail(1, "coefficient arrays missing");
  std::vector<std::string> nm;
  std::vector<double> val;
  for (int i = 0; i < nvalues; ++i) {
    if (!is_ident(names[i])) fail(1, "coefficient name %d is not an identifier", i);
    if (!std::isfinite(values[i])) fail(1, "coefficient '%s' is not finite", names[i]);
    if (!std::strcmp(names[i], "lap") || !std::strcmp(names[i], "bilap")) fail(1, "'%s' is reserved", names[i]);
    for (const std::string& o : nm)
      if (o == names[i]) fail(1, "coefficient '%s' given twice", names[i]);
    nm.push_back(names[i]);
    val.push_back(values[i]);
  }
  // statements and their left-hand sides first: a right-hand side may name
  // a field whose equation comes later
  std::vector<std::string> stmts;
  {
    std::string cur;
    for (const char* q = text;; ++q) {
      if (*q == ';' || *q == '\n' || *q == '\0') {
        bool blank = true;
        for (char ch : cur)
          if (!std::isspace((unsigned char)ch)) blank = false;
        if (!blank) stmts.push_back(cur);
        cur.clear();
        if (*q == '\0') break;
      } else {
        cur.push_back(*q);
      }
    }
  }
  if (stmts.empty()) fail(1, "no equation");
  if ((int)stmts.size() > EQ_MAX_FIELDS) fail(2, "%d fields: at most %d", (int)stmts.size(), EQ_MAX_FIELDS);
  const std::vector<std::string> none;
  const std::vector<double> nov;
  std::vector<std::string> fields;
  for (const std::string& st : stmts) {
    Reader r(st, none, none, nov);
    const std::string f = r.take_name();
    r.expect_op("'");
    if (!r.at_op("=")) fail(1, "each equation reads  name' = expression");
    if (f == "lap" || f == "bilap") fail(1, "'%s' is reserved", f.c_str());
    for (const std::string& o : fields)
      if (o == f) fail(1, "field '%s' has two equations", f.c_str());
    for (const std::string& o : nm)
      if (o == f) fail(1, "'%s' is both a field and a coefficient", f.c_str());
    fields.push_back(f);
  }
  std::memset(out, 0, sizeof(*out));
  out->nf = (int)fields.size();
  for (int j = 0; j < out->nf; ++j) {
    Reader r(stmts[j], fields, nm, val);
    r.take_name();
    r.expect_op("'");
    r.expect_op("=");
    Poly e = r.sum();
    if (r.kind() != T_END) fail(1, "trailing '%s' in the equation of '%s'", r.text().c_str(), fields[j].c_str());
    // L_psi: terms linear in field j itself; the symbol of lap^p is (-k^2)^p
    for (const Term& x : e.t) {
      if (!std::isfinite(x.c)) fail(1, "a coefficient of '%s' overflows", fields[j].c_str());
      const bool self = x.e[j] == 1 && x.e[1 - j] == 0;
      if (self) {
        if (x.p > EQ_MAX_LAP) fail(2, "'%s': L has lap^%d; lap^%d is the highest", fields[j].c_str(), x.p, EQ_MAX_LAP);
        out->L[j][x.p] += (x.p & 1) ? -x.c : x.c;
        continue;
      }
      // explicit (L_* or N): terms under the same derivative form one channel
      if (x.p > EQ_MAX_LAP)
        fail(2, "'%s': explicit terms under lap^%d; lap^%d is the highest", fields[j].c_str(), x.p, EQ_MAX_LAP);
      if (x.e[0] > EQ_MAX_EXP || x.e[1] > EQ_MAX_EXP)
        fail(2, "'%s': exponent above %d in an explicit term", fields[j].c_str(), EQ_MAX_EXP);
      int c = 0;
      while (c < out->nch[j] && out->ch[j][c].p != x.p) ++c;
      if (c == out->nch[j]) {
        if (c >= EQ_MAX_CH)
          fail(2, "'%s': explicit terms under more than %d derivatives", fields[j].c_str(), EQ_MAX_CH);
        out->ch[j][c].p = x.p;
        out->nch[j] = c + 1;
      }
      EqChannel& ch = out->ch[j][c];
      if (ch.nterm >= EQ_MAX_TERMS)
        fail(2, "'%s': more than %d explicit monomials under lap^%d", fields[j].c_str(), EQ_MAX_TERMS, x.p);
      ch.c[ch.nterm] = x.c;
      ch.e[ch.nterm][0] = x.e[0];
      ch.e[ch.nterm][1] = x.e[1];
      ch.nterm++;
    }
    // ascending derivative order
    if (out->nch[j] == 2 && out->ch[j][0].p > out->ch[j][1].p) std::swap(out->ch[j][0], out->ch[j][1]);
  }
}

}  // namespace

int eq_split(const char* text, const char* const names[], const double values[], int nvalues, EqSplit* out,
             char* msg, size_t msglen) {
  try {
    EqSplit tmp;
    split_all(text, names, values, nvalues, &tmp);
    *out = tmp;
    return 0;
  } catch (const Fail& f) {
    if (msg && msglen) snprintf(msg, msglen, "%s", f.msg.c_str());
    return f.code;
  } catch (...) {
    if (msg && msglen) snprintf(msg, msglen, "equation reader: internal error");
    return 1;
  }
}

}  // namespace ss
