// Runtime construction of the spectral scheme from equation text
// (Sec. 2.4.2): the tables one GPU step takes.  Host code only.
#pragma once

#include <stddef.h>

namespace ss {

constexpr int EQ_MAX_FIELDS = 2;
constexpr int EQ_MAX_CH = 2;       // explicit channels (distinct derivatives) of a field
constexpr int EQ_MAX_TERMS = 8;    // monomials of one channel
constexpr int EQ_MAX_EXP = 7;      // exponent of one field in a monomial
constexpr int EQ_MAX_LAP = 3;      // power of the Laplacian in L (L is cubic in k^2) and on a channel

// One explicit channel: the derivative lap^p (p = 0 .. 3) applied to
// E = sum_m c[m] f0^e[m][0] f1^e[m][1], m < nterm (the constant,
// other-field and nonlinear terms that share the derivative).
struct EqChannel {
  int p;
  int nterm;
  double c[EQ_MAX_TERMS];
  int e[EQ_MAX_TERMS][2];
};

// Result of the split for every field j:
//   L(k^2) = L[j][0] + L[j][1] k^2 + L[j][2] k^4 + L[j][3] k^6 (the symbol of
//   the terms linear in field j, lap -> -k^2), from which A;
//   nch[j] explicit channels ch[j][0 .. nch[j]-1], in ascending p.
struct EqSplit {
  int nf;
  double L[EQ_MAX_FIELDS][4];
  int nch[EQ_MAX_FIELDS];
  EqChannel ch[EQ_MAX_FIELDS][EQ_MAX_CH];
};

// Read and split the equations.  Returns 0 on success, else the ss_status
// code (1: the text or a name is invalid, 2: a valid equation outside the
// forms above) with a message in msg.
int eq_split(const char* text, const char* const names[], const double values[], int nvalues,
             EqSplit* out, char* msg, size_t msglen);

}  // namespace ss
