// Launch geometry and run-time dispatch of the templated kernels.
// The launch functions are instantiated once per element type in
// ss_kernels_f32.hip / ss_kernels_f64.hip.
#pragma once

#include "ss_kernels.hpp"

namespace ss {

template <typename T>
hipError_t run_xpass(int nx, int nf, int mode, int nlm, XArgs a, hipStream_t s);
template <typename T>
hipError_t run_ypass(int ny, int dir, YArgs a, int64_t nkx, hipStream_t s);
template <typename T>
hipError_t run_kpass(int nl, KArgs a, hipStream_t s);

#ifdef SS_DISPATCH_IMPL

template <typename T, int NX, int NF, int MODE, int NLM>
hipError_t launch_x(XArgs a, hipStream_t s) {
  typedef XCfg<T, NX> K;
  constexpr int RMAX = K::rmax(NF);
  const int R = (int)(a.rows < RMAX ? a.rows : RMAX);
  const int P = R / 2;
  int G = XThreads<T, NF>::value / K::S;
  if (G > P) G = P;
  if (G < 1) G = 1;
  a.rows_per_block = R;
  dim3 grid((unsigned)(a.rows / R)), block((unsigned)(G * K::S));
  hipLaunchKernelGGL((xpass_kernel<T, NX, NF, MODE, NLM>), grid, block, 0, s, a);
  return hipGetLastError();
}

#define SS_POW2_CASES(M) M(8) M(16) M(32) M(64) M(128) M(256) M(512) M(1024) M(2048) M(4096)

template <typename T, int NF, int MODE, int NLM>
hipError_t xdisp(int nx, const XArgs& a, hipStream_t s) {
  switch (nx) {
#define SS_CASE(n) \
  case n:          \
    return launch_x<T, n, NF, MODE, NLM>(a, s);
    SS_POW2_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_xpass(int nx, int nf, int mode, int nlm, XArgs a, hipStream_t s) {
  if (mode == XMODE_FWD) return xdisp<T, 1, XMODE_FWD, NLIN_POLY>(nx, a, s);
  if (mode == XMODE_INV) return xdisp<T, 1, XMODE_INV, NLIN_POLY>(nx, a, s);
  if (nf == 1) return xdisp<T, 1, XMODE_STEP, NLIN_POLY>(nx, a, s);
  if (nlm == NLIN_GS) return xdisp<T, 2, XMODE_STEP, NLIN_GS>(nx, a, s);
  return xdisp<T, 2, XMODE_STEP, NLIN_MODELC>(nx, a, s);
}

template <typename T, int NY, int DIR>
hipError_t launch_y(YArgs a, int64_t nkx, hipStream_t s) {
  typedef YCfg<T, NY> K;
  constexpr int RMAX = K::rmax();
  const int R = a.nz < RMAX ? a.nz : RMAX;
  int G = 1024 / K::S;
  if (G > R) G = R;
  if (G < 1) G = 1;
  a.lines_per_block = R;
  dim3 grid((unsigned)(nkx * (a.nz / R))), block((unsigned)(G * K::S));
  hipLaunchKernelGGL((ypass_kernel<T, NY, DIR>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t run_ypass(int ny, int dir, YArgs a, int64_t nkx, hipStream_t s) {
  switch (ny) {
#define SS_CASE(n)                                                       \
  case n:                                                                \
    return dir < 0 ? launch_y<T, n, -1>(a, nkx, s) : launch_y<T, n, +1>(a, nkx, s);
    SS_POW2_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

template <typename T, int NL>
hipError_t launch_k(KArgs a, hipStream_t s) {
  typedef KCfg<T, NL> K;
  const int L = a.nlines < K::LPW ? a.nlines : K::LPW;
  a.lines_per_block = L;
  dim3 grid((unsigned)(a.nlines / L), (unsigned)a.nf), block((unsigned)(L * K::S));
  hipLaunchKernelGGL((kpass_kernel<T, NL>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t run_kpass(int nl, KArgs a, hipStream_t s) {
  switch (nl) {
#define SS_CASE(n) \
  case n:          \
    return launch_k<T, n>(a, s);
    SS_POW2_CASES(SS_CASE)
#undef SS_CASE
  }
  return hipErrorInvalidValue;
}

#define SS_INSTANTIATE(T)                                                               \
  template hipError_t run_xpass<T>(int, int, int, int, XArgs, hipStream_t);            \
  template hipError_t run_ypass<T>(int, int, YArgs, int64_t, hipStream_t);             \
  template hipError_t run_kpass<T>(int, KArgs, hipStream_t);

#endif  // SS_DISPATCH_IMPL

}  // namespace ss
