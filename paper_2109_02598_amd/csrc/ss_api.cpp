// Host side of the C ABI declared in include/specstep.h.
//
// Sequencing per step (all on the grid's stream, no host synchronisation):
//   2D:  xpass STEP  (state -> psi -> f -> x-spectrum of f, scratch)
//        kpass       (y FFT of state and scratch, ETD1 update, inverse y FFT)
//   3D:  ypass INV   (state -> scratch: back to real y)
//        xpass STEP  (scratch in place: psi -> f -> x-spectrum of f)
//        ypass FWD   (scratch in place)
//        kpass       (z FFT, ETD1 update, inverse z FFT on the state)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/specstep.h"
#include "ss_dispatch.hpp"
#include "ss_equation.hpp"

namespace {

thread_local std::string g_err;

ss_status fail(ss_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ss_status fail(ss_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

ss_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(SS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return SS_OK;
}

bool pow2_in(int64_t v, int64_t lo, int64_t hi) {
  return v >= lo && v <= hi && (v & (v - 1)) == 0;
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct ss_grid_s {
  int ndim = 0;
  int64_t n[3] = {1, 1, 1};   // x, y, z
  double dx[3] = {1, 1, 1};
  ss_dtype dtype = SS_F64;
  hipStream_t stream = nullptr;

  bool has_model = false;
  ss_model model = SS_ALLEN_CAHN;
  int nf = 1;
  double coef[8] = {0};
  int ncoef = 0;
  double dt = 0;
  ss::KField kf[2];
  int nlm = ss::NLIN_POLY;
  double p[5] = {0};
  ss::NTab tab = {};   // explicit terms of equations read at run time (NLIN_TABLE), channel 0
  ss::NTab tab2 = {};  // the second explicit channel of each field (nsets = 2)
  int nsets = 1;       // x passes per step: 2 when a field has two explicit channels
  int scheme = 0;      // 0: ETD1 factors; 1: linearly implicit (ss_set_equations)
  ss::EqSplit eq = {};  // the split of ss_set_equations (finite-difference solver)

  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* state[2] = {nullptr, nullptr};
  void* scratch[2] = {nullptr, nullptr};
  void* staging = nullptr;
  void* shat[2] = {nullptr, nullptr};   // full spectrum of each field (stepping form)
  void* scratch2[2] = {nullptr, nullptr};   // second channel's nonlinear term (nsets = 2)
  // forward-Euler finite-difference solver (solver 1): real-space fields in
  // state[], the next step's in fd_next[], intermediates in fd_tmp[]
  int solver = 0;
  int stencil = 0;
  void* fd_next[2] = {nullptr, nullptr};
  void* fd_tmp[2] = {nullptr, nullptr};
  bool shat_valid = false;              // shat matches state
  bool field_set[2] = {false, false};

  double* mass_log = nullptr;
  int64_t log_cap = 0;
  int64_t log_count = 0;

  // tiling of each pass (rows or lines per workgroup); 0 = not chosen yet
  int tile_x_step = 0, tile_x_io = 0, tile_y = 0, tile_k = 0;
  int tile_x_ppb = 0;   // x pass tiles per block (> 1: persistent, prefetching)
  // arrays of a stepping-form step: 1 (default) every pass in place on the
  // state; 0 G in the scratch arrays, T back to the state; 2 G in the
  // scratch arrays and T over it, then state and scratch swap roles
  int step_arr = 1;
  bool step_arr_set = false;   // chosen by ss_set_step_arrangement: the tile cache leaves it alone
  // 0: the pass kernels (two launches per step); 1: one workgroup runs a
  // whole call of ss_step_n (small square one-field grids)
  int step_kind = 0;
  bool step_kind_set = false;  // chosen by ss_set_step_kernel: the tuner leaves it alone
  int lb = -1;          // log2 of the row block B of the spectral layout (-1: not chosen)

  // reverse mode: caller-owned workspace with checkpoints and segment
  void* adj_ws = nullptr;
  size_t adj_bytes = 0;
  int64_t adj_nsteps = 0;
  int adj_K = 0;
  bool adj_forward_done = false;
  double adj_coef[8] = {0};
  double adj_dt = 0;

  int64_t cells() const { return n[0] * n[1] * n[2]; }
  size_t esz() const { return (size_t)dtype; }
  size_t field_bytes() const { return (size_t)cells() * esz(); }
};

namespace {

int ncoef_of(ss_model m) {
  switch (m) {
    case SS_ALLEN_CAHN:
    case SS_CAHN_HILLIARD:
    case SS_PFC:
    case SS_GRAY_SCOTT:
      return 4;
    case SS_MODEL_C:
      return 5;
  }
  return -1;
}

// Linear symbol L(k^2) and operator N(k^2) of every field as polynomials
// in k^2, and the pointwise nonlinearity (the split of Eq. 1 written out
// for each model; every linear term, zeroth order included, is in L).
void build_operators(ss_grid g) {
  const double* c = g->coef;
  for (auto& f : g->kf) {
    for (double& v : f.l) v = 0;
    for (double& v : f.n) v = 0;
  }
  for (double& v : g->p) v = 0;
  switch (g->model) {
    case SS_ALLEN_CAHN: {  // M (kappa lap + c1) psi - M c2 psi^3
      const double M = c[0], kap = c[1], c1 = c[2], c2 = c[3];
      g->kf[0].l[0] = M * c1;
      g->kf[0].l[1] = -M * kap;
      g->kf[0].n[0] = -M * c2;
      g->nlm = ss::NLIN_POLY;
      g->p[0] = 0.0;
      g->p[1] = 1.0;
      break;
    }
    case SS_CAHN_HILLIARD: {  // M lap(c2 psi^3 - c1 psi - kappa lap psi)
      const double M = c[0], kap = c[1], c1 = c[2], c2 = c[3];
      g->kf[0].l[1] = M * c1;
      g->kf[0].l[2] = -M * kap;
      g->kf[0].n[1] = -M * c2;
      g->nlm = ss::NLIN_POLY;
      g->p[0] = 0.0;
      g->p[1] = 1.0;
      break;
    }
    case SS_PFC: {  // lap[(r + (q0^2 + lap)^2) psi + g2 psi^2 + g3 psi^3]
      const double r = c[0], q0 = c[1], g2 = c[2], g3 = c[3];
      const double q2 = q0 * q0;
      // -k^2 (r + (q0^2 - k^2)^2) = -(r + q0^4) k^2 + 2 q0^2 k^4 - k^6
      g->kf[0].l[1] = -(r + q2 * q2);
      g->kf[0].l[2] = 2.0 * q2;
      g->kf[0].l[3] = -1.0;
      g->kf[0].n[1] = -1.0;
      g->nlm = ss::NLIN_POLY;
      g->p[0] = g2;
      g->p[1] = g3;
      break;
    }
    case SS_GRAY_SCOTT: {  // u: Du lap - F, f = F - u v^2; v: Dv lap - (F+k), f = u v^2
      const double du = c[0], dv = c[1], F = c[2], kk = c[3];
      g->kf[0].l[0] = -F;
      g->kf[0].l[1] = -du;
      g->kf[0].n[0] = 1.0;
      g->kf[1].l[0] = -(F + kk);
      g->kf[1].l[1] = -dv;
      g->kf[1].n[0] = 1.0;
      g->nlm = ss::NLIN_GS;
      g->p[0] = F;
      break;
    }
    case SS_MODEL_C: {  // psi: c1 - k^2, f = -c2 psi^3 + 2 c5 psi m; m: c3 k^2 - k^4, N = k^2
      const double c1 = c[0], c2 = c[1], c3 = c[2], c4 = c[3], c5 = c[4];
      g->kf[0].l[0] = c1;
      g->kf[0].l[1] = -1.0;
      g->kf[0].n[0] = 1.0;
      g->kf[1].l[1] = c3;
      g->kf[1].l[2] = -1.0;
      g->kf[1].n[1] = 1.0;
      g->nlm = ss::NLIN_MODELC;
      g->p[0] = c2;
      g->p[1] = c4;
      g->p[2] = c5;
      break;
    }
    case SS_EQUATIONS:   // tables come from ss_set_equations
      break;
  }
}

void carve_workspace(ss_grid g) {
  char* b = (char*)g->ws;
  const size_t fb = align_up(g->field_bytes());
  if (g->solver == 1) {
    // state (nf), next (nf), two intermediates, staging
    for (int f = 0; f < 2; ++f) {
      g->state[f] = f < g->nf ? b + (size_t)f * fb : nullptr;
      g->fd_next[f] = f < g->nf ? b + (size_t)(g->nf + f) * fb : nullptr;
      g->scratch[f] = nullptr;
      g->shat[f] = nullptr;
    }
    g->fd_tmp[0] = b + (size_t)(2 * g->nf) * fb;
    g->fd_tmp[1] = b + (size_t)(2 * g->nf + 1) * fb;
    g->staging = b + (size_t)(2 * g->nf + 2) * fb;
    g->shat_valid = false;
    return;
  }
  for (int f = 0; f < 2; ++f) {
    g->state[f] = f < g->nf ? b + (size_t)f * fb : nullptr;
    g->scratch[f] = f < g->nf ? b + (size_t)(g->nf + f) * fb : nullptr;
  }
  g->staging = b + (size_t)(2 * g->nf) * fb;
  for (int f = 0; f < 2; ++f) g->shat[f] = f < g->nf ? b + (size_t)(2 * g->nf + 1 + f) * fb : nullptr;
  for (int f = 0; f < 2; ++f)
    g->scratch2[f] = (g->nsets == 2 && f < g->nf) ? b + (size_t)(3 * g->nf + 1 + f) * fb : nullptr;
  g->shat_valid = false;
}

// Optional per-launch timing: a pair of events is recorded around each
// kernel by the launch itself, so the pair brackets kernel time only.
struct PassTimer {
  enum { kMaxLaunches = 2048 };
  hipEvent_t ev[2 * kMaxLaunches];
  int kind[kMaxLaunches];
  int used = 0;
};

enum { PASS_X = 0, PASS_K = 1, PASS_YINV = 2, PASS_YFWD = 3 };

ss::LaunchEvents take_events(PassTimer* pt, int kind) {
  ss::LaunchEvents e;
  if (pt && pt->used < PassTimer::kMaxLaunches) {
    e.start = pt->ev[2 * pt->used];
    e.stop = pt->ev[2 * pt->used + 1];
    pt->kind[pt->used] = kind;
    pt->used++;
  }
  return e;
}

#define SS_TRY(x)                 \
  do {                            \
    ss_status st_ = (x);          \
    if (st_ != SS_OK) return st_; \
  } while (0)

// Tiles chosen by ss_autotune, shared by every grid of the same shape.
typedef std::tuple<int, int, int64_t, int64_t, int64_t, int> TileKey;  // ndim, esz, nx, ny, nz, nf
struct Tiles {
  int x_step, y, k, x_ppb, lb;
  int arr;   // step arrangement, -1: not chosen
};
std::mutex g_tile_mu;
std::map<TileKey, Tiles> g_tile_cache;

TileKey tile_key(ss_grid g) {
  return TileKey(g->ndim, (int)(2 * g->esz()), g->n[0], g->n[1], g->n[2], g->nf);
}

int esz_of(ss_grid g) { return (int)(2 * g->esz()); }
int64_t nlines_k(ss_grid g) { return (g->n[0] / 2) * (g->ndim == 3 ? g->n[1] : 1); }
int nlast(ss_grid g) { return (int)(g->ndim == 3 ? g->n[2] : g->n[1]); }

int ilog2i(int64_t v) {
  int l = 0;
  while ((int64_t(1) << (l + 1)) <= v) ++l;
  return l;
}

// Row block of the spectral layout: B rows of every kx stored together.
bool blk_ok(ss_grid g, int64_t B) {
  const int64_t rows = g->n[1] * g->n[2];
  if (!ss::is_pow2(B) || B > rows) return false;
  if (g->ndim == 3 && B > g->n[2]) return false;
  return true;
}
// The k-space pass reads a line in runs of B elements (one run per row
// block).  Runs shorter than a 128-byte L2 line leave the rest of the line
// to the neighbouring kx line, which usually runs on another XCD: each L2
// then fetches the whole line and the fabric carries up to twice the bytes
// (hidden by the Infinity Cache in time, not in traffic).  The default and
// the tuner's candidates therefore fill whole lines where the grid allows.
int64_t blk_default(ss_grid g) {
  int64_t B = 128 / esz_of(g);
  while (!blk_ok(g, B)) B /= 2;
  return B;
}

void ensure_tiles(ss_grid g) {
  const int esz = esz_of(g);
  if (!g->tile_x_io) g->tile_x_io = ss::x_tile_default(esz, (int)g->n[0], 1, g->n[1] * g->n[2]);
  if (g->lb >= 0 && g->tile_x_step && g->tile_k && (g->ndim == 2 || g->tile_y)) return;
  Tiles t = {0, 0, 0, 0, -1, -1};
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tile_cache.find(tile_key(g));
    if (it != g_tile_cache.end()) t = it->second;
  }
  if (g->lb < 0) g->lb = (t.lb >= 0 && !g->field_set[0]) ? t.lb : ilog2i(blk_default(g));
  if (!g->tile_x_step) {
    g->tile_x_step = t.x_step ? t.x_step : ss::x_tile_default(esz, (int)g->n[0], g->nf, g->n[1] * g->n[2]);
    g->tile_x_ppb = t.x_step ? t.x_ppb : 0;
  }
  if (!g->tile_k) g->tile_k = t.k ? t.k : ss::k_tile_default(esz, nlast(g), nlines_k(g), g->ndim == 3);
  if (g->ndim == 3 && !g->tile_y) g->tile_y = t.y ? t.y : ss::y_tile_default(esz, (int)g->n[1], g->n[2]);
  if (t.arr >= 0 && !g->step_arr_set) g->step_arr = t.arr;
}

// Coefficients of the x pass's pointwise terms (fixed models) or their
// monomial table (equations read at run time).
void fill_nonlinear(ss_grid g, ss::XArgs& a, int set = 0) {
  for (int i = 0; i < 5; ++i) a.p[i] = g->p[i];
  a.tab = set == 0 ? g->tab : g->tab2;
}

template <typename T>
ss_status launch_xpass(ss_grid g, int mode, int nf, const void* in0, const void* in1, void* out0,
                       void* out1, const void* real_in, void* real_out, double scale,
                       PassTimer* pt = nullptr, int nlm = -1, int set = 0) {
  ss::XArgs a;
  memset(&a, 0, sizeof(a));
  a.spec_in[0] = in0;
  a.spec_in[1] = in1;
  a.spec_out[0] = out0;
  a.spec_out[1] = out1;
  a.real_in = real_in;
  a.real_out = real_out;
  a.rows = g->n[1] * g->n[2];
  a.nz = (int)g->n[2];
  a.ny = (int)g->n[1];
  a.xcd_remap = 1;
  a.scale = scale;
  ensure_tiles(g);
  a.rows_per_block = (mode == ss::XMODE_STEP) ? g->tile_x_step : g->tile_x_io;
  a.tiles_per_block = (mode == ss::XMODE_STEP) ? g->tile_x_ppb : 0;
  a.lb = g->lb;
  fill_nonlinear(g, a, set);
  return hip_check(ss::run_xpass<T>((int)g->n[0], nf, mode, nlm >= 0 ? nlm : g->nlm, a, g->stream,
                                    take_events(pt, PASS_X)),
                   "x pass launch");
}

template <typename T>
ss_status launch_ypass(ss_grid g, int dir, const void* in, void* out, double scale,
                       PassTimer* pt = nullptr) {
  ss::YArgs a;
  memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.ny = (int)g->n[1];
  a.nz = (int)g->n[2];
  a.scale = scale;
  ensure_tiles(g);
  a.lines_per_block = g->tile_y;
  a.hx = (int)(g->n[0] / 2);
  a.lb = g->lb;
  return hip_check(ss::run_ypass<T>((int)g->n[1], dir, a, g->n[0] / 2, g->stream,
                                    take_events(pt, dir < 0 ? PASS_YFWD : PASS_YINV)),
                   "y pass launch");
}

// k-space pass of a step.  mode 1 (stepping form): S^ and G in, S^ and T
// out; mode 0: T and G in, T out (three transforms); mode 2: refresh S^
// from T.
template <typename T>
ss_status launch_kpass(ss_grid g, PassTimer* pt = nullptr, int mode = 1, int arr = 0) {
  ss::KArgs a;
  memset(&a, 0, sizeof(a));
  const bool three = g->ndim == 3;
  for (int f = 0; f < g->nf; ++f) {
    a.fld[f] = g->kf[f];
    a.fld[f].state = g->state[f];
    a.fld[f].nonlin = arr == 1 ? g->state[f] : g->scratch[f];   // G
    a.fld[f].out = arr == 2 ? g->scratch[f] : nullptr;           // T: over G, else to the state
    a.fld[f].shat = g->shat[f];
    a.fld[f].nonlin2 = (mode == 1 && g->nsets == 2) ? g->scratch2[f] : nullptr;
  }
  a.J = three ? (int)g->n[1] : 1;
  a.nlines = (int)(g->n[0] / 2) * a.J;
  a.nx = (int)g->n[0];
  const double two_pi = 6.283185307179586476925286766559;
  a.sx = two_pi / ((double)g->n[0] * g->dx[0]);
  a.sy = two_pi / ((double)g->n[1] * g->dx[1]);
  a.sz = three ? two_pi / ((double)g->n[2] * g->dx[2]) : 0.0;
  a.dt = g->dt;
  const int64_t nlast = three ? g->n[2] : g->n[1];
  a.a_scale = mode == 1 ? 1.0 : 1.0 / (double)nlast;
  a.b_scale = 1.0 / (double)g->cells();
  a.mass_log = mode == 2 ? nullptr : g->mass_log;
  a.log_index = g->log_count;
  a.log_capacity = g->log_cap;
  a.nf = g->nf;
  a.three_d = three ? 1 : 0;
  ensure_tiles(g);
  a.lines_per_block = g->tile_k;
  a.lb = g->lb;
  a.scheme = g->scheme;
  const int nl = (int)nlast;
  return hip_check(ss::run_kpass<T>(nl, a, mode, g->stream, mode == 2 ? ss::LaunchEvents() : take_events(pt, PASS_K)),
                   "k-space pass launch");
}

// Bring S^ up to date with the state (after the fields changed outside a
// stepping-form step).
template <typename T>
ss_status ensure_shat(ss_grid g) {
  if (g->shat_valid) return SS_OK;
  SS_TRY(launch_kpass<T>(g, nullptr, 2));
  g->shat_valid = true;
  return SS_OK;
}

// The one-workgroup step: 2D square grids N = 16 .. 128, one field, the
// fixed models' pointwise terms, ETD1 factors.
bool small_ok(ss_grid g) {
  return g->ndim == 2 && g->nf == 1 && g->solver == 0 && g->nlm == ss::NLIN_POLY && g->scheme == 0 &&
         g->n[0] == g->n[1] && ss::small_size_ok((int)g->n[0]);
}

// nsteps steps in one workgroup; the factor tables go to the scratch and
// staging arrays (free between the steps of the stepping form)
template <typename T>
ss_status small_run(ss_grid g, int64_t nsteps) {
  if (nsteps > 0x7fffffff) return fail(SS_ERR_ARG, "ss_step_n: too many steps for one run");
  ensure_tiles(g);
  ss::SmallArgs a;
  memset(&a, 0, sizeof(a));
  a.state = g->state[0];
  a.shat = g->shat[0];
  a.coef = g->scratch[0];
  a.coef_nyq = g->staging;
  a.lb = g->lb;
  a.nsteps = (int)nsteps;
  a.load_shat = g->shat_valid ? 1 : 0;
  const double two_pi = 6.283185307179586476925286766559;
  a.sx = two_pi / ((double)g->n[0] * g->dx[0]);
  a.sy = two_pi / ((double)g->n[1] * g->dx[1]);
  a.dt = g->dt;
  a.b_scale = 1.0 / (double)g->cells();
  a.f = g->kf[0];
  for (int i = 0; i < 3; ++i) a.p[i] = g->p[i];
  a.mass_log = g->mass_log;
  a.log_index = g->log_count;
  a.log_capacity = g->log_cap;
  SS_TRY(hip_check(ss::run_small<T>((int)g->n[0], a, g->stream), "one-workgroup step launch"));
  g->shat_valid = true;
  g->log_count += nsteps;
  return SS_OK;
}

// One step.  hat: the stepping form (S^ carried between steps; the caller
// has made it valid); otherwise the three-transform form, which leaves S^
// stale (the adjoint's checkpointed forward and its recomputation use it,
// so both follow the same arithmetic).
template <typename T>
ss_status step_once(ss_grid g, PassTimer* pt, bool hat = true) {
  // The stepping form can run every pass in place on the state arrays
  // (each workgroup reads its tile or lines whole before writing them; the
  // k-space pass writes T over G): a step then touches the state and its
  // spectrum only, which keeps more of them in the Infinity Cache.  Or G
  // goes to the scratch arrays and the k-space pass writes T over it, and
  // the two arrays swap roles.  The three-transform form reads T and G
  // together and keeps G in the scratch arrays.
  if (g->nsets == 2) {
    // two explicit channels: channel 1's terms go to scratch2 first, then
    // channel 0's over the state (2D) or into scratch (3D); the k-space
    // pass transforms both and writes T over channel 0's array
    if (!hat) return fail(SS_ERR_UNSUPPORTED, "two explicit channels: stepping form only");
    if (g->ndim == 2) {
      SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, g->nf, g->state[0], g->state[1], g->scratch2[0], g->scratch2[1],
                             nullptr, nullptr, 1.0, pt, -1, 1));
      SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, g->nf, g->state[0], g->state[1], g->state[0], g->state[1],
                             nullptr, nullptr, 1.0, pt, -1, 0));
      SS_TRY(launch_kpass<T>(g, pt, 1, 1));
    } else {
      for (int f = 0; f < g->nf; ++f) SS_TRY(launch_ypass<T>(g, +1, g->state[f], g->scratch[f], 1.0, pt));
      SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, g->nf, g->scratch[0], g->scratch[1], g->scratch2[0], g->scratch2[1],
                             nullptr, nullptr, 1.0, pt, -1, 1));
      SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, g->nf, g->scratch[0], g->scratch[1], g->scratch[0], g->scratch[1],
                             nullptr, nullptr, 1.0, pt, -1, 0));
      for (int f = 0; f < g->nf; ++f) {
        SS_TRY(launch_ypass<T>(g, -1, g->scratch2[f], g->scratch2[f], 1.0, pt));
        SS_TRY(launch_ypass<T>(g, -1, g->scratch[f], g->scratch[f], 1.0, pt));
      }
      SS_TRY(launch_kpass<T>(g, pt, 1, 0));
    }
    g->log_count++;
    return SS_OK;
  }
  const int arr = hat ? g->step_arr : 0;
  void** G = arr == 1 ? g->state : g->scratch;
  if (g->ndim == 2) {
    SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, g->nf, g->state[0], g->state[1], G[0], G[1], nullptr, nullptr,
                           1.0, pt));
  } else {
    for (int f = 0; f < g->nf; ++f) SS_TRY(launch_ypass<T>(g, +1, g->state[f], G[f], 1.0, pt));
    SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, g->nf, G[0], G[1], G[0], G[1], nullptr, nullptr, 1.0, pt));
    for (int f = 0; f < g->nf; ++f) SS_TRY(launch_ypass<T>(g, -1, G[f], G[f], 1.0, pt));
  }
  SS_TRY(launch_kpass<T>(g, pt, hat ? 1 : 0, arr));
  if (arr == 2)
    for (int f = 0; f < g->nf; ++f) std::swap(g->state[f], g->scratch[f]);
  if (!hat) g->shat_valid = false;
  g->log_count++;
  return SS_OK;
}

// ---- forward-Euler finite-difference step (Sec. 2.4.1, 2.2.2) -------------
// The kernels' stencil code: the axis-wise second-order stencil is 0 whether
// it was named by its point count (5 in 2D, 7 in 3D) or not.
int fd_kernel_stencil(ss_grid g) { return (g->stencil == 5 || g->stencil == 7) ? 0 : g->stencil; }

ss_status fd_launch(ss_grid g, int op, const void* in0, const void* in1, void* out0, void* out1, double s0) {
  ss::FDArgs a;
  memset(&a, 0, sizeof(a));
  a.in[0] = in0;
  a.in[1] = in1;
  a.out[0] = out0;
  a.out[1] = out1;
  a.nx = g->n[0];
  a.ny = g->n[1];
  a.nz = g->n[2];
  a.lx = ilog2i(g->n[0]);
  a.lxy = ilog2i(g->n[0] * g->n[1]);
  for (int d = 0; d < 3; ++d) a.ih2[d] = d < g->ndim ? 1.0 / (g->dx[d] * g->dx[d]) : 0.0;
  a.i6h2 = 1.0 / (6.0 * g->dx[0] * g->dx[0]);
  a.i30h2 = 1.0 / (30.0 * g->dx[0] * g->dx[0]);
  a.i12h2 = 1.0 / (12.0 * g->dx[0] * g->dx[0]);
  a.i60h2 = 1.0 / (60.0 * g->dx[0] * g->dx[0]);
  a.i120h2 = 1.0 / (120.0 * g->dx[0] * g->dx[0]);
  a.dt = g->dt;
  a.op = op;
  if (op == ss::FD_UPD) {
    a.p[0] = s0;
  } else {
    for (int i = 0; i < g->ncoef && i < 6; ++i) a.p[i] = g->coef[i];
  }
  const int st = fd_kernel_stencil(g);
  hipError_t e = g->dtype == SS_F64 ? ss::run_fd<double>(g->ndim, st, a, g->stream)
                                    : ss::run_fd<float>(g->ndim, st, a, g->stream);
  return hip_check(e, "finite-difference launch");
}

// Equations read at run time: field j's right-hand side as nested levels
// v_k = (-1)^k L[j][k] psi_j (+ E_j if p_j = k) + lap v_{k+1}, k = D_j .. 0
// (L is the symbol in k^2, and lap -> -k^2), one Laplacian a launch, from
// the top level down, alternating between the two intermediate arrays (a
// launch nesting two Laplacians recomputes too much to pay: its registers
// halve the occupancy); two fields with a single launch each share it.
ss_status fd_eq_launch(ss_grid g, const ss::FDEq& q, int depth) {
  ss::FDArgs a;
  memset(&a, 0, sizeof(a));
  a.in[0] = g->state[0];
  a.in[1] = g->nf > 1 ? g->state[1] : nullptr;
  a.nx = g->n[0];
  a.ny = g->n[1];
  a.nz = g->n[2];
  a.lx = ilog2i(g->n[0]);
  a.lxy = ilog2i(g->n[0] * g->n[1]);
  for (int d = 0; d < 3; ++d) a.ih2[d] = d < g->ndim ? 1.0 / (g->dx[d] * g->dx[d]) : 0.0;
  a.i6h2 = 1.0 / (6.0 * g->dx[0] * g->dx[0]);
  a.i30h2 = 1.0 / (30.0 * g->dx[0] * g->dx[0]);
  a.i12h2 = 1.0 / (12.0 * g->dx[0] * g->dx[0]);
  a.i60h2 = 1.0 / (60.0 * g->dx[0] * g->dx[0]);
  a.i120h2 = 1.0 / (120.0 * g->dx[0] * g->dx[0]);
  a.dt = g->dt;
  const int st = fd_kernel_stencil(g);
  hipError_t e = g->dtype == SS_F64 ? ss::run_fd_eq<double>(g->ndim, st, depth, a, q, g->stream)
                                    : ss::run_fd_eq<float>(g->ndim, st, depth, a, q, g->stream);
  return hip_check(e, "finite-difference launch");
}

// derivative of field j's explicit channel (-1: none; the finite-difference
// solver takes one channel per field)
int fd_eq_p(const ss::EqSplit& sp, int j) { return sp.nch[j] > 0 ? sp.ch[j][0].p : -1; }

int fd_eq_top(const ss::EqSplit& sp, int j) {
  int D = fd_eq_p(sp, j) > 0 ? fd_eq_p(sp, j) : 0;
  for (int k = 1; k < 4; ++k)
    if (sp.L[j][k] != 0.0) D = std::max(D, k);
  return D;
}

ss_status fd_eq_step(ss_grid g) {
  const ss::EqSplit& sp = g->eq;
  const int st = fd_kernel_stencil(g);
  ss::FDEq q;
  memset(&q, 0, sizeof(q));
  for (int j = 0; j < sp.nf; ++j) {
    q.tab.dv[j] = 0;
    const int nterm = sp.nch[j] > 0 ? sp.ch[j][0].nterm : 0;
    for (int m = 0; m < nterm; ++m) {
      const int e0 = sp.ch[j][0].e[m][0], e1 = sp.ch[j][0].e[m][1];
      q.tab.a[j][e1][e0] += sp.ch[j][0].c[m];
      q.tab.du[j][e1] = std::max(q.tab.du[j][e1], e0);
      q.tab.dv[j] = std::max(q.tab.dv[j], e1);
    }
    for (int k = 0; k < 8; ++k)
      for (int i = 0; i < 8; ++i) q.tab.af[j][k][i] = (float)q.tab.a[j][k][i];
  }
  // levels lo and hi = lo + depth of field j into slot s: v_lo computed,
  // v_hi from w (or pointwise when w is null)
  auto fill = [&](int s, int j, int lo, int depth, const void* w, void* out) {
    q.j[s] = j;
    for (int d = 0; d <= depth; ++d) {
      q.cl[s][d] = (lo + d) % 2 ? -sp.L[j][lo + d] : sp.L[j][lo + d];   // k^2 -> -lap
      q.el[s][d] = fd_eq_p(sp, j) == lo + d;
    }
    q.w[s] = w;
    q.out[s] = out;
  };
  // the wider stencils take E at the centre only: E at the top level then
  // gets a launch of its own
  auto own = [&](int j, int D) { return st != 0 && fd_eq_p(sp, j) == D && D > 0; };
  const int D0 = fd_eq_top(sp, 0), D1 = sp.nf > 1 ? fd_eq_top(sp, 1) : -1;
  if (sp.nf == 2 && D0 == D1 && D0 <= 1 && !own(0, D0) && !own(1, D1)) {
    q.nj = 2;
    q.fin = 1;
    fill(0, 0, 0, D0, nullptr, g->fd_next[0]);
    fill(1, 1, 0, D1, nullptr, g->fd_next[1]);
    SS_TRY(fd_eq_launch(g, q, D0));
  } else {
    for (int j = 0; j < sp.nf; ++j) {
      const int D = fd_eq_top(sp, j);
      int hi = D, t = 0;
      const void* w = nullptr;
      bool alone = own(j, D);
      while (true) {
        const int depth = (alone || hi == 0) ? 0 : 1;
        const int lo = hi - depth;
        alone = false;
        q.nj = 1;
        q.fin = lo == 0;
        void* out = lo == 0 ? g->fd_next[j] : g->fd_tmp[t];
        fill(0, j, lo, depth, w, out);
        SS_TRY(fd_eq_launch(g, q, depth));
        if (lo == 0) break;
        w = out;
        t ^= 1;
        hi = lo;
      }
    }
  }
  for (int f = 0; f < g->nf; ++f) std::swap(g->state[f], g->fd_next[f]);
  return SS_OK;
}

ss_status fd_step_once(ss_grid g) {
  if (g->model == SS_EQUATIONS) return fd_eq_step(g);
  void** S = g->state;
  void** N = g->fd_next;
  void** T = g->fd_tmp;
  const double* c = g->coef;
  switch (g->model) {
    case SS_ALLEN_CAHN:
      SS_TRY(fd_launch(g, ss::FD_AC, S[0], nullptr, N[0], nullptr, 0.0));
      break;
    case SS_GRAY_SCOTT:
      SS_TRY(fd_launch(g, ss::FD_GS, S[0], S[1], N[0], N[1], 0.0));
      break;
    case SS_CAHN_HILLIARD:
      // 2D axis-wise stencil on grids the row-marching kernel does not tile:
      // mu recomputed at the stencil points, one launch and two arrays (the
      // wider stencils recompute too much: 9 x 9 loads); where it tiles, its
      // two launches (mu, then the update) are faster
      if (g->ndim == 2 && (g->stencil == 0 || g->stencil == 5) &&
          (g->n[0] % ss::FD2_BX || g->n[1] % ss::FD2_YC)) {
        SS_TRY(fd_launch(g, ss::FD_CH, S[0], nullptr, N[0], nullptr, 0.0));
      } else {
        SS_TRY(fd_launch(g, ss::FD_MU_CH, S[0], nullptr, T[0], nullptr, 0.0));
        SS_TRY(fd_launch(g, ss::FD_UPD, S[0], T[0], N[0], nullptr, c[0]));
      }
      break;
    case SS_PFC:
      SS_TRY(fd_launch(g, ss::FD_LAP, S[0], nullptr, T[0], nullptr, 0.0));
      SS_TRY(fd_launch(g, ss::FD_MU_PFC, S[0], T[0], T[1], nullptr, 0.0));
      SS_TRY(fd_launch(g, ss::FD_UPD, S[0], T[1], N[0], nullptr, 1.0));
      break;
    default:  // model C
      SS_TRY(fd_launch(g, ss::FD_MC, S[0], S[1], N[0], T[0], 0.0));
      SS_TRY(fd_launch(g, ss::FD_UPD, S[1], T[0], N[1], nullptr, 1.0));
      break;
  }
  for (int f = 0; f < g->nf; ++f) std::swap(g->state[f], g->fd_next[f]);
  return SS_OK;
}

template <typename T>
ss_status set_field_t(ss_grid g, int field, const void* dsrc) {
  if (g->solver == 1)
    return hip_check(hipMemcpyAsync(g->state[field], dsrc, g->field_bytes(), hipMemcpyDeviceToDevice, g->stream),
                     "ss_set_field: copy");
  ss_status st = launch_xpass<T>(g, ss::XMODE_FWD, 1, nullptr, nullptr, g->state[field], nullptr,
                                 dsrc, nullptr, 1.0 / (double)g->n[0]);
  if (st != SS_OK) return st;
  if (g->ndim == 3)
    st = launch_ypass<T>(g, -1, g->state[field], g->state[field], 1.0 / (double)g->n[1]);
  return st;
}

template <typename T>
ss_status get_field_t(ss_grid g, int field, void* ddst) {
  if (g->solver == 1)
    return hip_check(hipMemcpyAsync(ddst, g->state[field], g->field_bytes(), hipMemcpyDeviceToDevice, g->stream),
                     "ss_get_field: copy");
  const void* spec = g->state[field];
  if (g->ndim == 3) {
    ss_status st = launch_ypass<T>(g, +1, g->state[field], g->scratch[field], 1.0);
    if (st != SS_OK) return st;
    spec = g->scratch[field];
  }
  return launch_xpass<T>(g, ss::XMODE_INV, 1, spec, nullptr, nullptr, nullptr, nullptr, ddst, 1.0);
}

// ---- structure factor (Sec. 3) ---------------------------------------------
// Number of radial bins: b = round(|m|) over the grid's integer mode vectors.
int sf_nbins(ss_grid g) {
  int64_t m2 = 0;
  for (int d = 0; d < g->ndim; ++d) m2 += (g->n[d] / 2) * (g->n[d] / 2);
  int64_t b = (int64_t)std::sqrt((double)m2);
  while (b * b + b < m2) ++b;
  while (b > 0 && b * b - b >= m2) --b;
  return (int)b + 1;
}

// |k| = 2 pi |m| / L needs the same box length along every axis
bool sf_isotropic(ss_grid g) {
  const double l0 = (double)g->n[0] * g->dx[0];
  for (int d = 1; d < g->ndim; ++d) {
    const double l = (double)g->n[d] * g->dx[d];
    if (std::fabs(l - l0) > 1e-12 * std::fabs(l0)) return false;
  }
  return true;
}

template <typename T>
ss_status sf_run(ss_grid g, int field, double* s_out, int64_t* n_out, int nbins) {
  const bool three = g->ndim == 3;
  void* rho = g->scratch[0];
  // occupancy spectrum: 3D inverse y first, then the x pass with the
  // threshold in place of f, then (3D) the forward y transform
  if (three) {
    SS_TRY(launch_ypass<T>(g, +1, g->state[field], rho, 1.0));
    SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, 1, rho, nullptr, rho, nullptr, nullptr, nullptr, 1.0, nullptr,
                           ss::NLIN_THRESH));
    SS_TRY(launch_ypass<T>(g, -1, rho, rho, 1.0));
  } else {
    SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, 1, g->state[field], nullptr, rho, nullptr, nullptr, nullptr, 1.0,
                           nullptr, ss::NLIN_THRESH));
  }
  ss::SFArgs a;
  memset(&a, 0, sizeof(a));
  a.spec = rho;
  a.nbins = nbins;
  a.J = three ? (int)g->n[1] : 1;
  a.nlines = (int)(g->n[0] / 2) * a.J;
  a.nx = (int)g->n[0];
  a.three_d = three ? 1 : 0;
  a.lb = g->lb;
  a.inv_n = 1.0 / (double)g->cells();
  const int nl = (int)(three ? g->n[2] : g->n[1]);
  const int esz = esz_of(g);
  ensure_tiles(g);
  int L = g->tile_k;
  while (L > (three ? 2 : 1) && !ss::sf_tile_ok(esz, nl, a.nlines, three, L, nbins)) L /= 2;
  if (!ss::sf_tile_ok(esz, nl, a.nlines, three, L, nbins))
    return fail(SS_ERR_UNSUPPORTED, "ss_structure_factor: no line tiling fits this grid");
  a.lines_per_block = L;
  // per-block partial histograms in the staging array
  a.pstride = (nbins + 31) & ~31;   // rows of whole 128-byte lines
  const int64_t per_block = (int64_t)a.pstride * (int64_t)(sizeof(double) + sizeof(uint32_t));
  const int64_t cap = (int64_t)g->field_bytes() / per_block;
  int64_t nblk = a.nlines / L;
  if (nblk > 512) nblk = 512;
  if (nblk > cap) nblk = cap;
  if (nblk < 1) return fail(SS_ERR_UNSUPPORTED, "ss_structure_factor: grid too small for %d bins", nbins);
  a.nblocks = (int)nblk;
  a.part_sum = (double*)g->staging;
  a.part_cnt = (uint32_t*)((char*)g->staging + (size_t)nblk * a.pstride * sizeof(double));
  a.s_out = s_out;
  a.n_out = n_out;
  SS_TRY(hip_check(ss::run_sfpass<T>(nl, a, g->stream), "structure factor pass launch"));
  return hip_check(ss::run_sfreduce<T>(a, g->stream), "structure factor reduce launch");
}

// Time one launch configuration: one warm-up launch, then `reps` launches
// each bracketed by its own events; returns the fastest in milliseconds.
template <typename F>
ss_status time_launch(ss_grid g, F launch, int reps, float* best_ms) {
  hipEvent_t e[2];
  SS_TRY(hip_check(hipEventCreate(&e[0]), "hipEventCreate"));
  ss_status st = hip_check(hipEventCreate(&e[1]), "hipEventCreate");
  if (st != SS_OK) {
    hipEventDestroy(e[0]);
    return st;
  }
  float best = 1e30f;
  st = launch(ss::LaunchEvents());
  for (int r = 0; st == SS_OK && r < reps; ++r) {
    ss::LaunchEvents ev;
    ev.start = e[0];
    ev.stop = e[1];
    st = launch(ev);
    if (st == SS_OK) st = hip_check(hipEventSynchronize(e[1]), "hipEventSynchronize");
    float ms = 0.f;
    if (st == SS_OK) st = hip_check(hipEventElapsedTime(&ms, e[0], e[1]), "hipEventElapsedTime");
    if (st == SS_OK && ms < best) best = ms;
  }
  hipEventDestroy(e[0]);
  hipEventDestroy(e[1]);
  *best_ms = best;
  return st;
}

// Tune the tiles of every pass for the current row block (g->lb); *total
// receives the summed best times of one step's launches.
template <typename T>
ss_status autotune_tiles(ss_grid g, int reps, float* total) {
  const int esz = esz_of(g);
  const int nx = (int)g->n[0];
  const int64_t rows = g->n[1] * g->n[2];
  float sum = 0.f;
  // while no field is stored the passes run on the step's own arrays (all
  // in place on the state); otherwise the fields are left alone
  const bool free_arrays = !g->field_set[0] && !g->field_set[1];
  // x pass (STEP): reads the state, writes it (free) or the scratch arrays
  {
    int best_r = 0, best_ppb = 0;
    float best = 1e30f;
    for (int r = 2; r <= 64; r *= 2)
      for (int ppb : {0, 2, 4, 8}) {
        if (!ss::x_tile_ok(esz, nx, g->nf, rows, r)) continue;
        if (ppb && !ss::x_pp_ok(esz, nx, g->nf, rows, r)) continue;
        if (ppb && rows / r < 2 * ppb) continue;
        auto launch = [&](ss::LaunchEvents ev) {
          ss::XArgs a;
          memset(&a, 0, sizeof(a));
          a.spec_in[0] = g->state[0];
          a.spec_in[1] = g->state[1];
          a.spec_out[0] = free_arrays ? g->state[0] : g->scratch[0];
          a.spec_out[1] = free_arrays ? g->state[1] : g->scratch[1];
          a.rows = rows;
          a.nz = (int)g->n[2];
          a.ny = (int)g->n[1];
          a.xcd_remap = 1;
          a.scale = 1.0;
          a.rows_per_block = r;
          a.tiles_per_block = ppb;
          a.lb = g->lb;
          fill_nonlinear(g, a);
          return hip_check(ss::run_xpass<T>(nx, g->nf, ss::XMODE_STEP, g->nlm, a, g->stream, ev), "autotune x");
        };
        float ms;
        SS_TRY(time_launch(g, launch, reps, &ms));
        if (ms < best) {
          best = ms;
          best_r = r;
          best_ppb = ppb;
        }
      }
    g->tile_x_step = best_r;
    g->tile_x_ppb = best_ppb;
    sum += best;
  }
  // k-space pass: while no field is stored, on the step's own arrays (the
  // traffic the step sees: S^, G -> S^, T over G); otherwise on the scratch
  // (as S^) and staging arrays, so the fields are untouched
  {
    const int nl = nlast(g);
    const int64_t nlines = nlines_k(g);
    int best_l = 0;
    float best = 1e30f;
    for (int l = 1; l <= 512; l *= 2) {
      if (!ss::k_tile_ok(esz, nl, nlines, g->ndim == 3, l)) continue;
      auto launch = [&](ss::LaunchEvents ev) {
        ss::KArgs a;
        memset(&a, 0, sizeof(a));
        // stepping form on the scratch (as S^) and staging (G in, T out,
        // per thread in place) arrays: the fields are untouched
        for (int f = 0; f < g->nf; ++f) {
          a.fld[f] = g->kf[f];
          if (free_arrays) {          // the step's own array roles (in place on the state)
            a.fld[f].shat = g->shat[f];
            a.fld[f].state = g->state[f];
            a.fld[f].nonlin = g->state[f];
          } else {
            a.fld[f].shat = g->scratch[f];
            a.fld[f].state = g->staging;
            a.fld[f].nonlin = g->staging;
          }
        }
        a.J = g->ndim == 3 ? (int)g->n[1] : 1;
        a.nlines = (int)nlines;
        a.nx = nx;
        const double two_pi = 6.283185307179586476925286766559;
        a.sx = two_pi / ((double)g->n[0] * g->dx[0]);
        a.sy = two_pi / ((double)g->n[1] * g->dx[1]);
        a.sz = g->ndim == 3 ? two_pi / ((double)g->n[2] * g->dx[2]) : 0.0;
        a.dt = g->dt;
        a.a_scale = 1.0;
        a.b_scale = 1.0 / (double)g->cells();
        a.nf = g->nf;
        a.scheme = g->scheme;
        a.three_d = g->ndim == 3;
        a.lines_per_block = l;
        a.lb = g->lb;
        return hip_check(ss::run_kpass<T>(nl, a, 1, g->stream, ev), "autotune k");
      };
      float ms;
      SS_TRY(time_launch(g, launch, reps, &ms));
      if (ms < best) {
        best = ms;
        best_l = l;
      }
    }
    g->tile_k = best_l;
    sum += best;
  }
  if (g->ndim == 3) {
    int best_y = 0;
    float best = 1e30f;
    for (int l = 1; l <= 64; l *= 2) {
      if (!ss::y_tile_ok(esz, (int)g->n[1], g->n[2], l)) continue;
      auto launch = [&](ss::LaunchEvents ev) {
        ss::YArgs a;
        memset(&a, 0, sizeof(a));
        a.in = free_arrays ? g->state[0] : g->scratch[0];
        a.out = free_arrays ? g->state[0] : g->scratch[0];
        a.ny = (int)g->n[1];
        a.nz = (int)g->n[2];
        a.hx = nx / 2;
        a.lb = g->lb;
        a.scale = 1.0;
        a.lines_per_block = l;
        return hip_check(ss::run_ypass<T>((int)g->n[1], -1, a, g->n[0] / 2, g->stream, ev), "autotune y");
      };
      float ms;
      SS_TRY(time_launch(g, launch, reps, &ms));
      if (ms < best) {
        best = ms;
        best_y = l;
      }
    }
    g->tile_y = best_y;
    sum += 2 * g->nf * best;   // one inverse and one forward y pass per field
  }
  *total = sum;
  return SS_OK;
}

// Mean time of one whole step on the step's own arrays, over n steps
// between two events (after one warm-up step).  Only while no field is
// stored: the contents are undefined; the mass log is detached.
template <typename T>
ss_status time_whole_steps(ss_grid g, int n, float* ms) {
  hipEvent_t e[2];
  SS_TRY(hip_check(hipEventCreate(&e[0]), "hipEventCreate"));
  ss_status st = hip_check(hipEventCreate(&e[1]), "hipEventCreate");
  if (st != SS_OK) {
    hipEventDestroy(e[0]);
    return st;
  }
  double* log = g->mass_log;
  const int64_t count = g->log_count;
  g->mass_log = nullptr;
  st = step_once<T>(g, nullptr, true);
  if (st == SS_OK) st = hip_check(hipEventRecord(e[0], g->stream), "hipEventRecord");
  for (int i = 0; st == SS_OK && i < n; ++i) st = step_once<T>(g, nullptr, true);
  if (st == SS_OK) st = hip_check(hipEventRecord(e[1], g->stream), "hipEventRecord");
  if (st == SS_OK) st = hip_check(hipEventSynchronize(e[1]), "hipEventSynchronize");
  float t = 0.f;
  if (st == SS_OK) st = hip_check(hipEventElapsedTime(&t, e[0], e[1]), "hipEventElapsedTime");
  g->mass_log = log;
  g->log_count = count;
  g->shat_valid = false;
  hipEventDestroy(e[0]);
  hipEventDestroy(e[1]);
  *ms = t / (float)n;
  return st;
}

// Whole-step time of the current tiling for the tuner: the better of two
// runs of 10*reps steps (candidates differ by 1-2%, about the spread of
// one short run).
template <typename T>
ss_status tune_steps(ss_grid g, int reps, float* ms) {
  float a, b;
  SS_TRY(time_whole_steps<T>(g, 10 * reps, &a));
  SS_TRY(time_whole_steps<T>(g, 10 * reps, &b));
  *ms = std::min(a, b);
  return SS_OK;
}

template <typename T>
ss_status autotune_t(ss_grid g, int reps) {
  // The row block of the layout can change only while no field is stored.
  const bool free_layout = !g->field_set[0] && !g->field_set[1];
  std::vector<int> lbs;
  if (free_layout) {
    const int64_t rows = g->n[1] * g->n[2];
    for (int64_t B : {blk_default(g), rows, (int64_t)64, (int64_t)32, (int64_t)16, (int64_t)8}) {
      if (!blk_ok(g, B) || B < blk_default(g)) continue;
      const int lb = ilog2i(B);
      if (std::find(lbs.begin(), lbs.end(), lb) == lbs.end()) lbs.push_back(lb);
    }
  } else {
    lbs.push_back(g->lb);
  }
  int best_lb = g->lb;
  int bx = 0, bppb = 0, bk = 0, by = 0;
  float best = 1e30f;
  for (int lb : lbs) {
    g->lb = lb;
    float tot;
    SS_TRY(autotune_tiles<T>(g, reps, &tot));
    // layouts compared by whole steps: the passes' per-launch times do not
    // see how one pass's writes meet the next one's reads
    if (lbs.size() > 1) SS_TRY(tune_steps<T>(g, reps, &tot));
    if (tot < best) {
      best = tot;
      best_lb = lb;
      bx = g->tile_x_step;
      bppb = g->tile_x_ppb;
      bk = g->tile_k;
      by = g->tile_y;
    }
  }
  g->lb = best_lb;
  g->tile_x_step = bx;
  g->tile_x_ppb = bppb;
  g->tile_k = bk;
  g->tile_y = by;
  if (free_layout) {
    // the arrays of a step (see step_once): fewer arrays in the caches
    // against the in-place x pass's access pattern (slower for FP32 in 2D)
    float best_arr = 1e30f;
    int barr = 1;
    for (int arr : {1, 0, 2}) {
      g->step_arr = arr;
      float ms;
      SS_TRY(tune_steps<T>(g, reps, &ms));
      if (ms < best_arr) {
        best_arr = ms;
        barr = arr;
      }
    }
    g->step_arr = barr;
    // the dominant pass's tiling, settled by whole steps as well: single
    // launches repeated on the same arrays can rank tilings differently
    // from steps once the arrays outgrow the Infinity Cache
    const int esz = esz_of(g);
    float best_step = 1e30f;
    for (int l = 1; l <= 512; l *= 2) {
      if (!ss::k_tile_ok(esz, nlast(g), nlines_k(g), g->ndim == 3, l)) continue;
      g->tile_k = l;
      float ms;
      SS_TRY(tune_steps<T>(g, reps, &ms));
      if (ms < best_step) {
        best_step = ms;
        bk = l;
      }
    }
    g->tile_k = bk;
    // then the x pass's tiling, the same way
    const int64_t rows = g->n[1] * g->n[2];
    const int nx = (int)g->n[0];
    best_step = 1e30f;
    for (int r = 2; r <= 64; r *= 2)
      for (int ppb : {0, 2, 4, 8}) {
        if (!ss::x_tile_ok(esz, nx, g->nf, rows, r)) continue;
        if (ppb && !ss::x_pp_ok(esz, nx, g->nf, rows, r)) continue;
        if (ppb && rows / r < 2 * ppb) continue;
        g->tile_x_step = r;
        g->tile_x_ppb = ppb;
        float ms;
        SS_TRY(tune_steps<T>(g, reps, &ms));
        if (ms < best_step) {
          best_step = ms;
          bx = r;
          bppb = ppb;
        }
      }
    g->tile_x_step = bx;
    g->tile_x_ppb = bppb;
    // small grids: the pass kernels against one workgroup running the steps
    if (small_ok(g) && !g->step_kind_set) {
      const int n = 10 * reps;
      float best_small = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        hipEvent_t e[2];
        SS_TRY(hip_check(hipEventCreate(&e[0]), "hipEventCreate"));
        SS_TRY(hip_check(hipEventCreate(&e[1]), "hipEventCreate"));
        double* log = g->mass_log;
        const int64_t count = g->log_count;
        g->mass_log = nullptr;
        ss_status st = hip_check(hipEventRecord(e[0], g->stream), "hipEventRecord");
        if (st == SS_OK) st = small_run<T>(g, n);
        if (st == SS_OK) st = hip_check(hipEventRecord(e[1], g->stream), "hipEventRecord");
        if (st == SS_OK) st = hip_check(hipEventSynchronize(e[1]), "hipEventSynchronize");
        float t = 0.f;
        if (st == SS_OK) st = hip_check(hipEventElapsedTime(&t, e[0], e[1]), "hipEventElapsedTime");
        g->mass_log = log;
        g->log_count = count;
        g->shat_valid = false;
        hipEventDestroy(e[0]);
        hipEventDestroy(e[1]);
        SS_TRY(st);
        best_small = std::min(best_small, t / (float)n);
      }
      g->step_kind = best_small < best_step ? 1 : 0;
    }
  }
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile_cache[tile_key(g)] = Tiles{g->tile_x_step, g->tile_y, g->tile_k, g->tile_x_ppb, g->lb,
                                     g->step_arr};
  return SS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batched step: grouped launches over many grids
// ---------------------------------------------------------------------------
struct ss_batch_s {
  std::vector<ss_grid> grids;
  std::vector<int> order;  // table order: largest grids first
  ss_dtype dtype = SS_F32;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int threads = 256;       // k-space launch; the x launch may use fewer
  int threads_x = 256;
  bool uploaded = false;
  std::vector<ss::BatchMember> table, table_tune;
  std::vector<void*> state_at_build;
  int x_total = 0, k_total = 0;
  uint32_t lds_x = 0, lds_k = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t graph_steps = 0;
  // 0: grouped launches (two per step); 1: one launch per run (a workgroup
  // per work item, ordered by a ticket counter); 2: one cooperative launch
  // per run (resident workgroups, two device-wide barriers a step)
  int mode = 0;
  int coop_blocks = 0;      // workgroups of the cooperative launch (0: not sized yet)
  bool coop_direct = false; // the captured run is the cooperative launch itself (no graph)
  bool mode_set = false;    // chosen by ss_batch_set_mode: the tuner leaves it alone
  unsigned spin_limit = 1u << 22;   // sleeps a wait of the single launch takes before it gives up
};

namespace {

bool batch_size_ok(int64_t n) { return n >= 64 && n <= 2048 && ss::is_pow2(n); }

// x-pass tile of one member for `tx` threads per block (0 if none)
int batch_x_rows(ss_grid g, int tx) {
  const int esz = esz_of(g);
  const int nx = (int)g->n[0], ny = (int)g->n[1];
  const bool sp = ss::x_small(esz, nx, 1, ny);
  const int R = 2 * tx / (nx / ss::x_pts_for(esz, nx, 1, sp));
  if (R < 2 || !ss::x_tile_ok(esz, nx, 1, ny, R) || ss::x_threads(esz, nx, 1, R, sp) != tx) return 0;
  return R;
}

// Member table for `threads` threads per k-space block; the x launch takes
// the largest power of two <= threads that tiles every member (16 points
// per thread make a small grid's rows short of threads).  False if a member
// cannot be tiled.
bool build_batch_table(ss_batch b, int threads, std::vector<ss::BatchMember>& tab,
                       std::vector<ss::BatchMember>& tune, int& x_total, int& k_total, uint32_t& lds_x,
                       uint32_t& lds_k, int& threads_x) {
  tab.clear();
  tune.clear();
  x_total = k_total = 0;
  lds_x = lds_k = 0;
  threads_x = threads;
  for (;;) {
    bool ok = true;
    for (int idx : b->order) ok = ok && batch_x_rows(b->grids[idx], threads_x) > 0;
    if (ok) break;
    threads_x /= 2;
    if (threads_x < 64) return false;
  }
  for (int idx : b->order) {
    ss_grid g = b->grids[idx];
    const int esz = esz_of(g);
    const int nx = (int)g->n[0], ny = (int)g->n[1];
    const int R = batch_x_rows(g, threads_x);
    const int L = threads / (ny / ss::k_pts(esz, ny));
    if (R < 2) return false;
    if (L < 1 || !ss::k_tile_ok(esz, ny, nx / 2, false, L)) return false;
    ss::BatchMember m;
    memset(&m, 0, sizeof(m));
    // in place on the state, as the single-grid step: two arrays per member
    // (T, S^) keep more of the batch in the Infinity Cache
    m.x.spec_in[0] = g->state[0];
    m.x.spec_out[0] = g->state[0];
    m.x.rows = ny;
    m.x.nz = 1;
    m.x.ny = ny;
    m.x.rows_per_block = R;
    m.x.xcd_remap = 0;
    m.x.scale = 1.0;
    ensure_tiles(g);
    m.x.lb = g->lb;
    for (int i = 0; i < 5; ++i) m.x.p[i] = g->p[i];
    m.k.fld[0] = g->kf[0];
    m.k.fld[0].state = g->state[0];
    m.k.fld[0].nonlin = g->state[0];
    m.k.fld[0].shat = g->shat[0];
    m.k.nlines = nx / 2;
    m.k.J = 1;
    m.k.lines_per_block = L;
    m.k.nx = nx;
    const double two_pi = 6.283185307179586476925286766559;
    m.k.sx = two_pi / ((double)nx * g->dx[0]);
    m.k.sy = two_pi / ((double)ny * g->dx[1]);
    m.k.dt = g->dt;
    m.k.a_scale = 1.0;   // stepping form
    m.k.b_scale = 1.0 / (double)g->cells();
    m.k.nf = 1;
    m.k.lb = g->lb;
    m.nx = nx;
    m.ny = ny;
    m.xsp = ss::x_small(esz, nx, 1, ny) ? 1 : 0;   // as the plain path's x pass
    m.x_first = x_total;
    m.x_tiles = ny / R;
    m.k_first = k_total;
    m.k_tiles = (nx / 2) / L;
    x_total += m.x_tiles;
    k_total += m.k_tiles;
    const uint32_t lx = (uint32_t)ss::x_lds(esz, nx, 1, R), lk = (uint32_t)ss::k_lds(esz, ny, L);
    if (lx > lds_x) lds_x = lx;
    if (lk > lds_k) lds_k = lk;
    tab.push_back(m);
    // tuning copy, which leaves the fields alone: the x pass writes the
    // scratch array; the k pass runs on the scratch (as S^) and staging (G
    // in, T out) arrays
    m.x.spec_out[0] = g->scratch[0];
    m.k.fld[0].shat = g->scratch[0];
    m.k.fld[0].state = g->staging;
    m.k.fld[0].nonlin = g->staging;
    tune.push_back(m);
  }
  return true;
}

size_t batch_table_bytes(ss_batch b) { return align_up(sizeof(ss::BatchMember) * b->grids.size()); }
// after the two tables: ticket and error flag, then per-member counters
size_t batch_sync_bytes(ss_batch b) { return align_up(sizeof(unsigned) * (2 + 2 * b->grids.size())); }

ss::BatchSync batch_sync(ss_batch b, int64_t nsteps) {
  ss::BatchSync y;
  unsigned* base = (unsigned*)((char*)b->ws + 2 * batch_table_bytes(b));
  y.ctl = base;
  y.xdone = base + 2;
  y.kdone = base + 2 + b->grids.size();
  y.nsteps = (int)nsteps;
  y.spin_limit = b->spin_limit;
  return y;
}

// The single launch needs one block size for both passes.
bool batch_single_ok(ss_batch b) { return b->uploaded && b->threads_x == b->threads; }

// Steps one launch can hold: a workgroup per work item, and the dispatch
// counts work-items (threads) in 32 bits.
int64_t batch_single_max_steps(ss_batch b) {
  const int64_t per_step = (int64_t)(b->x_total + b->k_total) * b->threads;
  return std::max<int64_t>(1, (int64_t)0xffffffffLL / per_step);
}

ss_status batch_upload(ss_batch b, int threads) {
  if (!build_batch_table(b, threads, b->table, b->table_tune, b->x_total, b->k_total, b->lds_x, b->lds_k,
                         b->threads_x))
    return fail(SS_ERR_UNSUPPORTED, "batch: a member cannot be tiled with %d threads per block", threads);
  const size_t tb = batch_table_bytes(b);
  SS_TRY(hip_check(hipMemcpyAsync(b->ws, b->table.data(), sizeof(ss::BatchMember) * b->table.size(),
                                  hipMemcpyHostToDevice, b->stream), "batch table upload"));
  SS_TRY(hip_check(hipMemcpyAsync((char*)b->ws + tb, b->table_tune.data(),
                                  sizeof(ss::BatchMember) * b->table_tune.size(), hipMemcpyHostToDevice, b->stream),
                   "batch table upload"));
  SS_TRY(hip_check(hipStreamSynchronize(b->stream), "batch table upload"));
  b->threads = threads;
  b->uploaded = true;
  b->coop_blocks = 0;
  b->state_at_build.clear();
  for (ss_grid g : b->grids) b->state_at_build.push_back(g->state[0]);
  return SS_OK;
}

ss_status batch_check_members(ss_batch b) {
  for (size_t i = 0; i < b->grids.size(); ++i) {
    ss_grid g = b->grids[i];
    if (!g->ws || !g->field_set[0]) return fail(SS_ERR_STATE, "batch member %zu: workspace or field not set", i);
    if (b->uploaded && b->state_at_build[i] != g->state[0])
      return fail(SS_ERR_STATE, "batch member %zu: workspace was rebound after the batch table was built", i);
  }
  return SS_OK;
}

// Bring every member's S^ up to date, on the batch's stream.
ss_status batch_refresh(ss_batch b) {
  for (ss_grid g : b->grids) {
    if (g->shat_valid) continue;
    hipStream_t own = g->stream;
    g->stream = b->stream;
    ss_status st = g->dtype == SS_F64 ? ensure_shat<double>(g) : ensure_shat<float>(g);
    g->stream = own;
    SS_TRY(st);
  }
  return SS_OK;
}

template <typename T>
ss_status batch_launch_step(ss_batch b, bool tune_table, ss::LaunchEvents evx, ss::LaunchEvents evk) {
  ss::BatchArgs a;
  a.m = (const ss::BatchMember*)((char*)b->ws + (tune_table ? batch_table_bytes(b) : 0));
  a.count = (int)b->grids.size();
  a.x_total = b->x_total;
  a.k_total = b->k_total;
  SS_TRY(hip_check(ss::run_batch_x<T>(a, b->threads_x, b->x_total, b->lds_x, b->stream, evx), "batch x launch"));
  return hip_check(ss::run_batch_k<T>(a, b->threads, b->k_total, b->lds_k, b->stream, evk), "batch k launch");
}

ss_status batch_step_once(ss_batch b) {
  return b->dtype == SS_F64 ? batch_launch_step<double>(b, false, {}, {}) : batch_launch_step<float>(b, false, {}, {});
}

// nsteps steps of every member in one launch (after the reset of its
// counters): one workgroup per work item.
template <typename T>
ss_status batch_launch_single(ss_batch b, int64_t nsteps, bool tune_table, ss::LaunchEvents ev) {
  if (!batch_single_ok(b))
    return fail(SS_ERR_UNSUPPORTED, "batch: the single launch needs one block size for both passes");
  if (nsteps < 1 || nsteps > batch_single_max_steps(b))
    return fail(SS_ERR_ARG, "batch: %lld steps do not fit one launch", (long long)nsteps);
  ss::BatchArgs a;
  a.m = (const ss::BatchMember*)((char*)b->ws + (tune_table ? batch_table_bytes(b) : 0));
  a.count = (int)b->grids.size();
  a.x_total = b->x_total;
  a.k_total = b->k_total;
  return hip_check(ss::run_batch_single<T>(a, batch_sync(b, nsteps), b->threads,
                                           std::max(b->lds_x, b->lds_k), b->stream, ev),
                   "batch single launch");
}

// Workgroups of the cooperative launch: as many as are resident at once,
// at most one per tile of the larger pass.
template <typename T>
ss_status batch_coop_size(ss_batch b) {
  int fit = 0;
  SS_TRY(hip_check(ss::run_batch_coop<T>(ss::BatchArgs(), ss::BatchSync(), b->threads, std::max(b->lds_x, b->lds_k), 0,
                                         &fit, b->stream, {}),
                   "batch: cooperative occupancy"));
  b->coop_blocks = std::min(fit, std::max(b->x_total, b->k_total));
  if (b->coop_blocks < 1) return fail(SS_ERR_UNSUPPORTED, "batch: no workgroup of the cooperative launch fits a CU");
  return SS_OK;
}

// Steps one cooperative launch can hold: its barrier counter (two arrivals
// per workgroup and step) counts in 32 bits.
int64_t batch_coop_max_steps(ss_batch b) {
  return std::max<int64_t>(1, (int64_t)0xffffffffLL / (2 * (int64_t)std::max(b->coop_blocks, 1)) - 1);
}

template <typename T>
ss_status batch_launch_coop(ss_batch b, int64_t nsteps, bool tune_table, ss::LaunchEvents ev) {
  if (!batch_single_ok(b))
    return fail(SS_ERR_UNSUPPORTED, "batch: the cooperative launch needs one block size for both passes");
  if (!b->coop_blocks) SS_TRY(batch_coop_size<T>(b));
  if (nsteps < 1 || nsteps > batch_coop_max_steps(b))
    return fail(SS_ERR_ARG, "batch: %lld steps do not fit one launch", (long long)nsteps);
  ss::BatchArgs a;
  a.m = (const ss::BatchMember*)((char*)b->ws + (tune_table ? batch_table_bytes(b) : 0));
  a.count = (int)b->grids.size();
  a.x_total = b->x_total;
  a.k_total = b->k_total;
  return hip_check(ss::run_batch_coop<T>(a, batch_sync(b, nsteps), b->threads, std::max(b->lds_x, b->lds_k),
                                         b->coop_blocks, nullptr, b->stream, ev),
                   "batch cooperative launch");
}

// Synchronise the batch's stream and report a single launch whose bounded
// wait ran out.
ss_status batch_check_error(ss_batch b) {
  if (!b->ws) return SS_OK;
  unsigned flag = 0;
  SS_TRY(hip_check(hipMemcpyAsync(&flag, batch_sync(b, 1).ctl + 1, sizeof(flag), hipMemcpyDeviceToHost, b->stream),
                   "batch: error flag copy"));
  SS_TRY(hip_check(hipStreamSynchronize(b->stream), "batch: synchronise"));
  if (flag) return fail(SS_ERR_DEVICE, "batch: a single launch gave up waiting for a member's tiles");
  return SS_OK;
}

ss_status batch_run(ss_batch b, int64_t nsteps) {
  if (nsteps < 1) return SS_OK;
  if (b->mode == 2) {
    for (int64_t done = 0; done < nsteps;) {
      if (!b->coop_blocks)
        SS_TRY(b->dtype == SS_F64 ? batch_coop_size<double>(b) : batch_coop_size<float>(b));
      const int64_t n = std::min(nsteps - done, batch_coop_max_steps(b));
      SS_TRY(b->dtype == SS_F64 ? batch_launch_coop<double>(b, n, false, {})
                                : batch_launch_coop<float>(b, n, false, {}));
      done += n;
    }
    return SS_OK;
  }
  if (b->mode == 1) {
    // one launch, or several in a row when the steps exceed one launch's size
    for (int64_t done = 0; done < nsteps;) {
      const int64_t n = std::min(nsteps - done, batch_single_max_steps(b));
      SS_TRY(b->dtype == SS_F64 ? batch_launch_single<double>(b, n, false, {})
                                : batch_launch_single<float>(b, n, false, {}));
      done += n;
    }
    return SS_OK;
  }
  for (int64_t i = 0; i < nsteps; ++i) SS_TRY(batch_step_once(b));
  return SS_OK;
}

}  // namespace


// ---------------------------------------------------------------------------
// Reverse mode (Gray-Scott, 2D)
// ---------------------------------------------------------------------------
namespace {

struct AdjLayout {
  size_t fb;            // one field array
  int64_t nck;          // checkpoints
  size_t ckpt, segT, segG, lam, la, mu, acc, dc, total;
};

AdjLayout adj_layout(ss_grid g, int64_t nsteps, int K) {
  AdjLayout L;
  L.fb = align_up(g->field_bytes());
  L.nck = (nsteps + K - 1) / K;
  size_t o = 0;
  L.ckpt = o; o += (size_t)L.nck * 2 * L.fb;
  L.segT = o; o += (size_t)K * 2 * L.fb;
  L.segG = o; o += (size_t)K * 2 * L.fb;
  L.lam = o; o += 2 * L.fb;
  L.la = o; o += 2 * L.fb;
  L.mu = o; o += 2 * L.fb;
  L.acc = o; o += align_up(sizeof(double) * 2 * 2 * (size_t)(g->n[0] / 2));
  L.dc = o; o += align_up(sizeof(double));
  L.total = o;
  return L;
}

char* adj_ptr(ss_grid g, size_t off) { return (char*)g->adj_ws + off; }
void* ck_field(ss_grid g, const AdjLayout& L, int64_t i, int f) { return adj_ptr(g, L.ckpt + ((size_t)i * 2 + f) * L.fb); }
void* seg_T(ss_grid g, const AdjLayout& L, int64_t j, int f) { return adj_ptr(g, L.segT + ((size_t)j * 2 + f) * L.fb); }
void* seg_G(ss_grid g, const AdjLayout& L, int64_t j, int f) { return adj_ptr(g, L.segG + ((size_t)j * 2 + f) * L.fb); }

template <typename T>
ss_status kpass_to(ss_grid g, const void* st0, const void* st1, const void* g0, const void* g1, void* o0, void* o1) {
  ss::KArgs a;
  memset(&a, 0, sizeof(a));
  const void* st[2] = {st0, st1};
  const void* gn[2] = {g0, g1};
  void* out[2] = {o0, o1};
  for (int f = 0; f < 2; ++f) {
    a.fld[f] = g->kf[f];
    a.fld[f].state = const_cast<void*>(st[f]);
    a.fld[f].nonlin = gn[f];
    a.fld[f].out = out[f];
  }
  a.J = 1;
  a.nlines = (int)(g->n[0] / 2);
  a.nx = (int)g->n[0];
  const double two_pi = 6.283185307179586476925286766559;
  a.sx = two_pi / ((double)g->n[0] * g->dx[0]);
  a.sy = two_pi / ((double)g->n[1] * g->dx[1]);
  a.dt = g->dt;
  a.a_scale = 1.0 / (double)g->n[1];
  a.b_scale = 1.0 / (double)g->cells();
  a.nf = 2;
  ensure_tiles(g);
  a.lines_per_block = g->tile_k;
  a.lb = g->lb;
  return hip_check(ss::run_kpass<T>((int)g->n[1], a, 0, g->stream, ss::LaunchEvents()), "k-space pass launch");
}

template <typename T>
ss_status adjoint_t(ss_grid g, const void* const dqT[], void* const dq0[], double* dcoef) {
  const AdjLayout L = adj_layout(g, g->adj_nsteps, g->adj_K);
  const int64_t nsteps = g->adj_nsteps;
  const int K = g->adj_K;
  const int esz = esz_of(g);
  const int nx = (int)g->n[0], ny = (int)g->n[1];
  void* lam[2] = {adj_ptr(g, L.lam), adj_ptr(g, L.lam + L.fb)};
  void* la[2] = {adj_ptr(g, L.la), adj_ptr(g, L.la + L.fb)};
  void* mu[2] = {adj_ptr(g, L.mu), adj_ptr(g, L.mu + L.fb)};
  double* acc = (double*)adj_ptr(g, L.acc);
  double* dc = (double*)adj_ptr(g, L.dc);
  const int kl = ss::kadj_tile(ny, nx / 2);
  const int kblocks = (nx / 2) / kl;
  SS_TRY(hip_check(hipMemsetAsync(acc, 0, sizeof(double) * 2 * 2 * kblocks, g->stream), "hipMemsetAsync"));
  SS_TRY(hip_check(hipMemsetAsync(dc, 0, sizeof(double), g->stream), "hipMemsetAsync"));
  // lambda^T = dJ/dq^T, in the spectral state layout
  for (int f = 0; f < 2; ++f)
    SS_TRY(launch_xpass<T>(g, ss::XMODE_FWD, 1, nullptr, nullptr, lam[f], nullptr, dqT[f], nullptr,
                           1.0 / (double)nx));
  ss::KAdjArgs ka;
  memset(&ka, 0, sizeof(ka));
  for (int f = 0; f < 2; ++f) {
    ka.fld[f].lam = lam[f];
    ka.fld[f].out_a = la[f];
    ka.fld[f].out_m = mu[f];
    ka.fld[f].l[0] = g->kf[f].l[0];
    ka.fld[f].l[1] = g->kf[f].l[1];
  }
  ka.nlines = nx / 2;
  ka.lines_per_block = kl;
  ka.nx = nx;
  const double two_pi = 6.283185307179586476925286766559;
  ka.sx = two_pi / ((double)nx * g->dx[0]);
  ka.sy = two_pi / ((double)ny * g->dx[1]);
  ka.dt = g->dt;
  ka.a_scale = 1.0 / (double)ny;
  ka.nxd = (double)nx;
  ka.acc = acc;
  ka.dc = dc;
  ensure_tiles(g);
  ka.lb = g->lb;
  ss::XAdjArgs xa;
  memset(&xa, 0, sizeof(xa));
  for (int f = 0; f < 2; ++f) {
    xa.m[f] = mu[f];
    xa.la[f] = la[f];
    xa.out[f] = lam[f];
  }
  xa.rows = ny;
  xa.lb = g->lb;
  xa.rows_per_block = ss::xadj_tile(esz, nx, ny);
  if (!xa.rows_per_block) return fail(SS_ERR_UNSUPPORTED, "ss_adjoint_n: grid too large for the adjoint x pass");
  const int64_t nseg = L.nck;
  for (int64_t sgi = nseg - 1; sgi >= 0; --sgi) {
    const int64_t s0 = sgi * K;
    const int64_t s1 = (s0 + K < nsteps) ? s0 + K : nsteps;
    // recompute the segment: states q^n and nonlinear terms g^n, n in [s0, s1)
    for (int f = 0; f < 2; ++f)
      SS_TRY(hip_check(hipMemcpyAsync(seg_T(g, L, 0, f), ck_field(g, L, sgi, f), g->field_bytes(),
                                      hipMemcpyDeviceToDevice, g->stream), "checkpoint copy"));
    for (int64_t n = s0; n < s1; ++n) {
      const int64_t j = n - s0;
      SS_TRY(launch_xpass<T>(g, ss::XMODE_STEP, 2, seg_T(g, L, j, 0), seg_T(g, L, j, 1), seg_G(g, L, j, 0),
                             seg_G(g, L, j, 1), nullptr, nullptr, 1.0));
      if (n + 1 < s1)
        SS_TRY(kpass_to<T>(g, seg_T(g, L, j, 0), seg_T(g, L, j, 1), seg_G(g, L, j, 0), seg_G(g, L, j, 1),
                           seg_T(g, L, j + 1, 0), seg_T(g, L, j + 1, 1)));
    }
    // sweep the segment backwards
    for (int64_t n = s1 - 1; n >= s0; --n) {
      const int64_t j = n - s0;
      for (int f = 0; f < 2; ++f) {
        ka.fld[f].q = seg_T(g, L, j, f);
        ka.fld[f].g = seg_G(g, L, j, f);
        xa.q[f] = seg_T(g, L, j, f);
      }
      SS_TRY(hip_check(ss::run_kadj<T>(ny, ka, g->stream), "adjoint k-space launch"));
      SS_TRY(hip_check(ss::run_xadj<T>(nx, xa, g->stream), "adjoint x launch"));
    }
  }
  for (int f = 0; f < 2; ++f)
    SS_TRY(launch_xpass<T>(g, ss::XMODE_INV, 1, lam[f], nullptr, nullptr, nullptr, nullptr, dq0[f], 1.0));
  std::vector<double> hacc((size_t)2 * 2 * kblocks);
  double hdc = 0;
  SS_TRY(hip_check(hipMemcpyAsync(hacc.data(), acc, sizeof(double) * hacc.size(), hipMemcpyDeviceToHost, g->stream),
                   "gradient copy"));
  SS_TRY(hip_check(hipMemcpyAsync(&hdc, dc, sizeof(double), hipMemcpyDeviceToHost, g->stream), "gradient copy"));
  SS_TRY(hip_check(hipStreamSynchronize(g->stream), "ss_adjoint_n: synchronise"));
  double S0[2] = {0, 0}, S1[2] = {0, 0};
  for (int f = 0; f < 2; ++f)
    for (int b = 0; b < kblocks; ++b) {
      S0[f] += hacc[2 * ((size_t)f * kblocks + b)];
      S1[f] += hacc[2 * ((size_t)f * kblocks + b) + 1];
    }
  // S_j = Nx * acc_j (the kernel sums w (Nx dA P' + dB Q') with P' and Q'
  // built from the /Nx-scaled spectra); inner products carry 1/N.
  const double scale = (double)nx / (double)g->cells();
  dcoef[0] = -S1[0] * scale;                              // Du: dL_u/dDu = -k^2
  dcoef[1] = -S1[1] * scale;                              // Dv: dL_v/dDv = -k^2
  dcoef[2] = -(S0[0] + S0[1]) * scale + hdc;              // F: dL/dF = -1 (both), dg_u/dF = 1
  dcoef[3] = -S0[1] * scale;                              // k: dL_v/dk = -1
  return SS_OK;
}

}  // namespace

namespace {

bool finite_all(const double* v, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

namespace {

// Launch one pass of the current tiling for timing.  While no field is
// stored, every pass runs as in a step, in place on the state arrays.
// Otherwise in a form that leaves the fields alone: the x pass reads the
// state and writes the scratch arrays; the k-space pass runs on the
// scratch arrays with the staging array as nonlinear term and output, in
// place; the y passes run in place on scratch 0.  The in-place forms touch fewer distinct arrays than a step,
// so where the step's arrays outgrow the Infinity Cache they can read fast.
template <typename T>
ss_status launch_timed_pass(ss_grid g, int pass, ss::LaunchEvents ev) {
  const bool free_arrays = !g->field_set[0] && !g->field_set[1];
  const int nx = (int)g->n[0];
  const int64_t rows = g->n[1] * g->n[2];
  if (pass == PASS_X) {
    ss::XArgs a;
    memset(&a, 0, sizeof(a));
    a.spec_in[0] = g->state[0];
    a.spec_in[1] = g->state[1];
    a.spec_out[0] = free_arrays ? g->state[0] : g->scratch[0];
    a.spec_out[1] = free_arrays ? g->state[1] : g->scratch[1];
    a.rows = rows;
    a.nz = (int)g->n[2];
    a.ny = (int)g->n[1];
    a.xcd_remap = 1;
    a.scale = 1.0;
    a.rows_per_block = g->tile_x_step;
    a.tiles_per_block = g->tile_x_ppb;
    a.lb = g->lb;
    fill_nonlinear(g, a);
    return hip_check(ss::run_xpass<T>(nx, g->nf, ss::XMODE_STEP, g->nlm, a, g->stream, ev), "timed x pass");
  }
  if (pass == PASS_K) {
    const int nl = nlast(g);
    ss::KArgs a;
    memset(&a, 0, sizeof(a));
    for (int f = 0; f < g->nf; ++f) {
      a.fld[f] = g->kf[f];
      if (free_arrays) {
        a.fld[f].shat = g->shat[f];
        a.fld[f].state = g->state[f];
        a.fld[f].nonlin = g->state[f];
      } else {
        a.fld[f].shat = g->scratch[f];
        a.fld[f].state = g->staging;
        a.fld[f].nonlin = g->staging;
      }
    }
    a.J = g->ndim == 3 ? (int)g->n[1] : 1;
    a.nlines = (int)nlines_k(g);
    a.nx = nx;
    const double two_pi = 6.283185307179586476925286766559;
    a.sx = two_pi / ((double)g->n[0] * g->dx[0]);
    a.sy = two_pi / ((double)g->n[1] * g->dx[1]);
    a.sz = g->ndim == 3 ? two_pi / ((double)g->n[2] * g->dx[2]) : 0.0;
    a.dt = g->dt;
    a.a_scale = 1.0;
    a.b_scale = 1.0 / (double)g->cells();
    a.nf = g->nf;
    a.scheme = g->scheme;
    a.three_d = g->ndim == 3;
    a.lines_per_block = g->tile_k;
    a.lb = g->lb;
    return hip_check(ss::run_kpass<T>(nl, a, 1, g->stream, ev), "timed k pass");
  }
  if (g->ndim == 3 && (pass == PASS_YINV || pass == PASS_YFWD)) {
    ss::YArgs a;
    memset(&a, 0, sizeof(a));
    a.in = free_arrays ? g->state[0] : g->scratch[0];   // a step: in place on the state
    a.out = free_arrays ? g->state[0] : g->scratch[0];
    a.ny = (int)g->n[1];
    a.nz = (int)g->n[2];
    a.scale = 1.0;
    a.lines_per_block = g->tile_y;
    a.hx = (int)(g->n[0] / 2);
    a.lb = g->lb;
    return hip_check(ss::run_ypass<T>((int)g->n[1], pass == PASS_YFWD ? -1 : +1, a, g->n[0] / 2, g->stream, ev),
                     "timed y pass");
  }
  return fail(SS_ERR_ARG, "ss_time_pass: pass %d does not exist for this grid", pass);
}

}  // namespace

extern "C" {

const char* ss_last_error(void) { return g_err.c_str(); }

const char* ss_version(void) { return "specstep 0.1 gfx950"; }

ss_status ss_create_grid(int ndim, const int64_t n[], const double dx[], ss_dtype dtype,
                         void* stream, ss_grid* out) {
  if (!out) return fail(SS_ERR_ARG, "ss_create_grid: out is null");
  *out = nullptr;
  if (!n || !dx) return fail(SS_ERR_ARG, "ss_create_grid: n or dx is null");
  if (ndim != 2 && ndim != 3) return fail(SS_ERR_ARG, "ss_create_grid: ndim must be 2 or 3, got %d", ndim);
  if (dtype != SS_F32 && dtype != SS_F64) return fail(SS_ERR_ARG, "ss_create_grid: dtype must be SS_F32 or SS_F64");
  for (int d = 0; d < ndim; ++d) {
    if (!(std::isfinite(dx[d]) && dx[d] > 0.0))
      return fail(SS_ERR_ARG, "ss_create_grid: dx[%d] must be finite and > 0", d);
    if (!pow2_in(n[d], 8, 4096))
      return fail(SS_ERR_UNSUPPORTED, "ss_create_grid: n[%d] = %lld is not a power of two in [8, 4096]", d,
                  (long long)n[d]);
  }
  if (ndim == 3 && n[2] > 1024)
    return fail(SS_ERR_UNSUPPORTED, "ss_create_grid: 3D grids need n[2] <= 1024");
  ss_grid g = new (std::nothrow) ss_grid_s();
  if (!g) return fail(SS_ERR_ARG, "ss_create_grid: out of host memory");
  g->ndim = ndim;
  for (int d = 0; d < ndim; ++d) {
    g->n[d] = n[d];
    g->dx[d] = dx[d];
  }
  g->dtype = dtype;
  g->stream = (hipStream_t)stream;
  *out = g;
  return SS_OK;
}

ss_status ss_set_model(ss_grid g, ss_model model, const double* coef, int ncoef, double dt) {
  if (!g) return fail(SS_ERR_ARG, "ss_set_model: null grid");
  if (model == SS_EQUATIONS) return fail(SS_ERR_ARG, "ss_set_model: equations are set with ss_set_equations");
  const int want = ncoef_of(model);
  if (want < 0) return fail(SS_ERR_ARG, "ss_set_model: unknown model %d", (int)model);
  if (ncoef != want) return fail(SS_ERR_ARG, "ss_set_model: model %d takes %d coefficients, got %d", (int)model, want, ncoef);
  if (!coef) return fail(SS_ERR_ARG, "ss_set_model: coef is null");
  if (!finite_all(coef, ncoef)) return fail(SS_ERR_ARG, "ss_set_model: non-finite coefficient");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(SS_ERR_ARG, "ss_set_model: dt must be finite and > 0");
  const int nf = (model == SS_GRAY_SCOTT || model == SS_MODEL_C) ? 2 : 1;
  if (g->has_model && model != g->model) {
    g->ws = nullptr;
    g->ws_bytes = 0;
    g->field_set[0] = g->field_set[1] = false;
  }
  if (!g->has_model || nf != g->nf) g->tile_x_step = g->tile_y = g->tile_k = 0;
  if (g->has_model && model != g->model) g->lb = -1;
  g->model = model;
  g->nf = nf;
  g->ncoef = ncoef;
  for (int i = 0; i < ncoef; ++i) g->coef[i] = coef[i];
  g->dt = dt;
  g->has_model = true;
  g->scheme = 0;
  g->nsets = 1;
  build_operators(g);
  return SS_OK;
}

namespace {

// Largest value of L(k^2) = l0 + l1 k^2 + l2 k^4 + l3 k^6 over k^2 in
// [0, kmax2]: the ends and the stationary points inside.
double max_symbol(const double* l, double kmax2) {
  auto L = [&](double q) { return l[0] + q * (l[1] + q * (l[2] + q * l[3])); };
  double best = std::max(L(0.0), L(kmax2));
  // L'(q) = l1 + 2 l2 q + 3 l3 q^2
  const double a = 3.0 * l[3], b = 2.0 * l[2], c = l[1];
  std::vector<double> roots;
  if (a == 0.0) {
    if (b != 0.0) roots.push_back(-c / b);
  } else {
    const double disc = b * b - 4.0 * a * c;
    if (disc >= 0.0) {
      const double sq = std::sqrt(disc);
      roots.push_back((-b + sq) / (2.0 * a));
      roots.push_back((-b - sq) / (2.0 * a));
    }
  }
  for (double q : roots)
    if (q > 0.0 && q < kmax2) best = std::max(best, L(q));
  return best;
}

}  // namespace

ss_status ss_split_equations(const char* equations, const char* const names[], const double values[],
                             int nvalues, double* out, int nout) {
  if (!out || nout < SS_SPLIT_OUT_LEN) return fail(SS_ERR_ARG, "ss_split_equations: out needs %d doubles", SS_SPLIT_OUT_LEN);
  ss::EqSplit sp;
  char msg[256];
  const int rc = ss::eq_split(equations, names, values, nvalues, &sp, msg, sizeof(msg));
  if (rc) return fail((ss_status)rc, "ss_split_equations: %s", msg);
  for (int i = 0; i < SS_SPLIT_OUT_LEN; ++i) out[i] = 0.0;
  out[0] = sp.nf;
  for (int j = 0; j < sp.nf; ++j) {
    double* o = out + 1 + SS_SPLIT_FIELD_LEN * j;
    for (int i = 0; i < 4; ++i) o[i] = sp.L[j][i];
    o[4] = sp.nch[j];
    for (int c = 0; c < sp.nch[j]; ++c) {
      const ss::EqChannel& ch = sp.ch[j][c];
      double* q = o + 5 + SS_SPLIT_CHANNEL_LEN * c;
      q[0] = ch.p;
      q[1] = ch.nterm;
      for (int m = 0; m < ch.nterm; ++m) {
        q[2 + 3 * m] = ch.c[m];
        q[3 + 3 * m] = ch.e[m][0];
        q[4 + 3 * m] = ch.e[m][1];
      }
    }
  }
  return SS_OK;
}

ss_status ss_set_equations(ss_grid g, const char* equations, const char* const names[], const double values[],
                           int nvalues, double dt, int scheme) {
  if (!g) return fail(SS_ERR_ARG, "ss_set_equations: null grid");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(SS_ERR_ARG, "ss_set_equations: dt must be finite and > 0");
  if (scheme != 0 && scheme != 1) return fail(SS_ERR_ARG, "ss_set_equations: unknown scheme %d", scheme);
  if (g->solver == 1 && scheme != 0)
    return fail(SS_ERR_UNSUPPORTED, "ss_set_equations: the finite-difference solver is explicit (scheme 0)");
  ss::EqSplit sp;
  char msg[256];
  const int rc = ss::eq_split(equations, names, values, nvalues, &sp, msg, sizeof(msg));
  if (rc) return fail((ss_status)rc, "ss_set_equations: %s", msg);
  ss::KField kf[2];
  ss::NTab tab;
  memset(kf, 0, sizeof(kf));
  memset(&tab, 0, sizeof(tab));
  double kmax2 = 0.0;
  for (int d = 0; d < g->ndim; ++d) kmax2 += (M_PI / g->dx[d]) * (M_PI / g->dx[d]);
  ss::NTab tab2;
  memset(&tab2, 0, sizeof(tab2));
  int nsets = 1;
  for (int j = 0; j < sp.nf; ++j) nsets = std::max(nsets, sp.nch[j]);
  if (nsets == 2 && g->solver == 1)
    return fail(SS_ERR_UNSUPPORTED, "ss_set_equations: the finite-difference solver takes one explicit channel per field");
  for (int j = 0; j < sp.nf; ++j) {
    for (int i = 0; i < 4; ++i) kf[j].l[i] = sp.L[j][i];
    for (int c = 0; c < sp.nch[j]; ++c) {
      const ss::EqChannel& ch = sp.ch[j][c];
      double* n = c == 0 ? kf[j].n : kf[j].n2;
      n[ch.p] = (ch.p & 1) ? -1.0 : 1.0;   // lap^p -> (-k^2)^p
      // monomials -> dense table: a[j][power of field 1][power of field 0]
      ss::NTab& t = c == 0 ? tab : tab2;
      for (int m = 0; m < ch.nterm; ++m) {
        const int e0 = ch.e[m][0], e1 = ch.e[m][1];
        t.a[j][e1][e0] += ch.c[m];
        t.du[j][e1] = std::max(t.du[j][e1], e0);
        t.dv[j] = std::max(t.dv[j], e1);
      }
    }
    for (int k = 0; k < 8; ++k)
      for (int i = 0; i < 8; ++i) {
        tab.af[j][k][i] = (float)tab.a[j][k][i];
        tab2.af[j][k][i] = (float)tab2.a[j][k][i];
      }
    if (scheme == 1 && !(max_symbol(kf[j].l, kmax2) * dt < 1.0))
      return fail(SS_ERR_ARG, "ss_set_equations: 1 - L dt is not positive for every mode of field %d", j);
  }
  const bool same = g->has_model && g->model == SS_EQUATIONS && g->nf == sp.nf && g->nsets == nsets;
  if (g->has_model && !same) {
    g->ws = nullptr;
    g->ws_bytes = 0;
    g->field_set[0] = g->field_set[1] = false;
  }
  if (!g->has_model || sp.nf != g->nf) g->tile_x_step = g->tile_y = g->tile_k = 0;
  if (g->has_model && g->model != SS_EQUATIONS) g->lb = -1;
  g->model = SS_EQUATIONS;
  g->nf = sp.nf;
  g->ncoef = 0;
  g->dt = dt;
  g->scheme = scheme;
  for (double& v : g->p) v = 0;
  g->kf[0] = kf[0];
  g->kf[1] = kf[1];
  g->tab = tab;
  g->tab2 = tab2;
  g->nsets = nsets;
  g->eq = sp;
  g->nlm = ss::NLIN_TABLE;
  g->has_model = true;
  return SS_OK;
}

ss_status ss_workspace_size(ss_grid g, size_t* bytes) {
  if (!g || !bytes) return fail(SS_ERR_ARG, "ss_workspace_size: null argument");
  if (!g->has_model) return fail(SS_ERR_STATE, "ss_workspace_size: call ss_set_model first");
  *bytes = align_up(g->field_bytes()) *
           (size_t)(g->solver == 1 ? 2 * g->nf + 3 : 3 * g->nf + 1 + (g->nsets == 2 ? g->nf : 0));
  return SS_OK;
}

ss_status ss_get_step_arrangement(ss_grid g, int* arr) {
  if (!g || !arr) return fail(SS_ERR_ARG, "ss_get_step_arrangement: null argument");
  *arr = g->step_arr;
  return SS_OK;
}

ss_status ss_set_step_arrangement(ss_grid g, int arr) {
  if (!g) return fail(SS_ERR_ARG, "ss_set_step_arrangement: null grid");
  if (arr < 0 || arr > 2) return fail(SS_ERR_ARG, "ss_set_step_arrangement: arrangement %d is not 0, 1 or 2", arr);
  g->step_arr = arr;
  g->step_arr_set = true;
  return SS_OK;
}

ss_status ss_set_step_kernel(ss_grid g, int kind) {
  if (!g) return fail(SS_ERR_ARG, "ss_set_step_kernel: null grid");
  if (kind != 0 && kind != 1) return fail(SS_ERR_ARG, "ss_set_step_kernel: kind %d is not 0 or 1", kind);
  if (kind == 1 && !g->has_model) return fail(SS_ERR_STATE, "ss_set_step_kernel: call ss_set_model first");
  if (kind == 1 && !small_ok(g))
    return fail(SS_ERR_UNSUPPORTED,
                "ss_set_step_kernel: one workgroup takes 2D square one-field grids of 16 to 128 points a side, "
                "the fixed models, spectral solver");
  g->step_kind = kind;
  g->step_kind_set = true;
  return SS_OK;
}

ss_status ss_get_step_kernel(ss_grid g, int* kind) {
  if (!g || !kind) return fail(SS_ERR_ARG, "ss_get_step_kernel: null argument");
  *kind = (g->step_kind == 1 && small_ok(g)) ? 1 : 0;
  return SS_OK;
}

ss_status ss_set_solver(ss_grid g, int solver, int stencil) {
  if (!g) return fail(SS_ERR_ARG, "ss_set_solver: null grid");
  if (solver != 0 && solver != 1) return fail(SS_ERR_ARG, "ss_set_solver: unknown solver %d", solver);
  if (solver == 1 && g->has_model && g->model == SS_EQUATIONS && g->scheme != 0)
    return fail(SS_ERR_UNSUPPORTED, "ss_set_solver: the finite-difference solver is explicit (scheme 0)");
  if (solver == 1 && g->has_model && g->model == SS_EQUATIONS && g->nsets != 1)
    return fail(SS_ERR_UNSUPPORTED, "ss_set_solver: the finite-difference solver takes one explicit channel per field");
  if (solver == 1) {
    const bool ok = stencil == 0 || stencil == 4 ||
                    (g->ndim == 2 ? (stencil == 5 || stencil == 9 || stencil == 17 || stencil == 21)
                                  : (stencil == 7 || stencil == 15 || stencil == 19 || stencil == 21 || stencil == 27));
    if (!ok) return fail(SS_ERR_ARG, "ss_set_solver: stencil %d is not available in %dD", stencil, g->ndim);
    if (stencil != 0 && stencil != 4 && stencil != 5 && stencil != 7)
      for (int d = 1; d < g->ndim; ++d)
        if (std::fabs(g->dx[d] - g->dx[0]) > 1e-12 * g->dx[0])
          return fail(SS_ERR_UNSUPPORTED, "ss_set_solver: the isotropic stencil needs equal spacings");
  } else if (stencil != 0) {
    return fail(SS_ERR_ARG, "ss_set_solver: the spectral solver takes no stencil");
  }
  if (solver != g->solver) {
    g->ws = nullptr;
    g->ws_bytes = 0;
    g->field_set[0] = g->field_set[1] = false;
  }
  g->solver = solver;
  g->stencil = stencil;
  return SS_OK;
}

ss_status ss_bind_workspace(ss_grid g, void* device_ptr, size_t bytes) {
  if (!g) return fail(SS_ERR_ARG, "ss_bind_workspace: null grid");
  if (!g->has_model) return fail(SS_ERR_STATE, "ss_bind_workspace: call ss_set_model first");
  size_t need = 0;
  ss_workspace_size(g, &need);
  if (!device_ptr) return fail(SS_ERR_ARG, "ss_bind_workspace: null pointer");
  if (((uintptr_t)device_ptr) % kAlign) return fail(SS_ERR_ARG, "ss_bind_workspace: pointer not 256-byte aligned");
  if (bytes < need) return fail(SS_ERR_ARG, "ss_bind_workspace: %zu bytes given, %zu needed", bytes, need);
  if (device_ptr != g->ws) g->field_set[0] = g->field_set[1] = false;
  g->ws = device_ptr;
  g->ws_bytes = bytes;
  carve_workspace(g);
  return SS_OK;
}

ss_status ss_set_field(ss_grid g, int field, const void* src, int src_on_device) {
  if (!g) return fail(SS_ERR_ARG, "ss_set_field: null grid");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_set_field: model and workspace must be set first");
  if (field < 0 || field >= g->nf) return fail(SS_ERR_ARG, "ss_set_field: field %d out of range [0, %d)", field, g->nf);
  if (!src) return fail(SS_ERR_ARG, "ss_set_field: src is null");
  const void* dsrc = src;
  ss_status st;
  if (!src_on_device) {
    st = hip_check(hipMemcpyAsync(g->staging, src, g->field_bytes(), hipMemcpyHostToDevice, g->stream),
                   "ss_set_field: host to device copy");
    if (st != SS_OK) return st;
    dsrc = g->staging;
  }
  st = g->dtype == SS_F64 ? set_field_t<double>(g, field, dsrc) : set_field_t<float>(g, field, dsrc);
  if (st != SS_OK) return st;
  if (!src_on_device) {
    st = hip_check(hipStreamSynchronize(g->stream), "ss_set_field: synchronise");
    if (st != SS_OK) return st;
  }
  g->field_set[field] = true;
  g->shat_valid = false;
  return SS_OK;
}

ss_status ss_get_field(ss_grid g, int field, void* dst, int dst_on_device) {
  if (!g) return fail(SS_ERR_ARG, "ss_get_field: null grid");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_get_field: model and workspace must be set first");
  if (field < 0 || field >= g->nf) return fail(SS_ERR_ARG, "ss_get_field: field %d out of range [0, %d)", field, g->nf);
  if (!g->field_set[field]) return fail(SS_ERR_STATE, "ss_get_field: field %d was never set", field);
  if (!dst) return fail(SS_ERR_ARG, "ss_get_field: dst is null");
  void* ddst = dst_on_device ? dst : g->staging;
  ss_status st = g->dtype == SS_F64 ? get_field_t<double>(g, field, ddst) : get_field_t<float>(g, field, ddst);
  if (st != SS_OK) return st;
  if (!dst_on_device) {
    st = hip_check(hipMemcpyAsync(dst, g->staging, g->field_bytes(), hipMemcpyDeviceToHost, g->stream),
                   "ss_get_field: device to host copy");
    if (st != SS_OK) return st;
    st = hip_check(hipStreamSynchronize(g->stream), "ss_get_field: synchronise");
    if (st != SS_OK) return st;
  }
  return SS_OK;
}

ss_status ss_step_n(ss_grid g, int64_t nsteps) {
  if (!g) return fail(SS_ERR_ARG, "ss_step_n: null grid");
  if (nsteps < 0) return fail(SS_ERR_ARG, "ss_step_n: nsteps must be >= 0");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_step_n: model and workspace must be set first");
  for (int f = 0; f < g->nf; ++f)
    if (!g->field_set[f]) return fail(SS_ERR_STATE, "ss_step_n: field %d was never set", f);
  if (g->solver == 1) {
    for (int64_t i = 0; i < nsteps; ++i) SS_TRY(fd_step_once(g));
    return SS_OK;
  }
  if (nsteps > 0 && g->step_kind == 1 && small_ok(g))
    return g->dtype == SS_F64 ? small_run<double>(g, nsteps) : small_run<float>(g, nsteps);
  if (nsteps > 0) SS_TRY(g->dtype == SS_F64 ? ensure_shat<double>(g) : ensure_shat<float>(g));
  for (int64_t i = 0; i < nsteps; ++i) {
    ss_status st = g->dtype == SS_F64 ? step_once<double>(g, nullptr) : step_once<float>(g, nullptr);
    if (st != SS_OK) return st;
  }
  return SS_OK;
}

}  // extern "C"

// ---- stepping without allocation --------------------------------------------
// The arrays of ss_step_fields_noalloc live in one fixed device array of
// the library (each GPU the library runs on holds its own copy, allocated
// when the code object loads, until the process ends).  In host code the
// name is only a stand-in: kernels and copies take the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SS_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
ss_status scratch_for_current_device(void** out) {
  int dev = -1;
  SS_TRY(hip_check(hipGetDevice(&dev), "ss_step_fields_noalloc: current device"));
  if (dev < 0 || dev >= kMaxDevices) return fail(SS_ERR_DEVICE, "ss_step_fields_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    SS_TRY(hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "ss_step_fields_noalloc: address of the scratch array"));
    if (!p || ((uintptr_t)p) % kAlign) return fail(SS_ERR_DEVICE, "ss_step_fields_noalloc: scratch array misplaced");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SS_OK;
}

// Arrays a no-allocation call carves from the fixed array: the state and
// its spectrum (2 nf), and with two explicit channels the second channel's
// terms (nf) and, in 3D, the real-y arrays the x passes read (nf).
size_t noalloc_arrays(ss_grid g) {
  size_t n = 2 * (size_t)g->nf;
  if (g->nsets == 2) n += (size_t)g->nf * (g->ndim == 3 ? 2 : 1);
  return n;
}

// set_field + step_n + get_field with the state and its spectrum carved
// from `base` and every pass in place; the grid's own arrays and flags are
// put back afterwards.
template <typename T>
ss_status step_fields_t(ss_grid g, void* const fields[], int64_t nsteps, char* base) {
  const size_t fb = align_up(g->field_bytes());
  void* keep_state[2] = {g->state[0], g->state[1]};
  void* keep_scratch[2] = {g->scratch[0], g->scratch[1]};
  void* keep_shat[2] = {g->shat[0], g->shat[1]};
  void* keep_scratch2[2] = {g->scratch2[0], g->scratch2[1]};
  void* keep_staging = g->staging;
  const bool keep_valid = g->shat_valid;
  const int keep_arr = g->step_arr;
  for (int f = 0; f < 2; ++f) {
    g->state[f] = f < g->nf ? base + (size_t)f * fb : nullptr;
    g->scratch[f] = g->state[f];   // 3D read-out: inverse y pass in place
    g->shat[f] = f < g->nf ? base + (size_t)(g->nf + f) * fb : nullptr;
    g->scratch2[f] = nullptr;
    if (g->nsets == 2 && f < g->nf) {
      g->scratch2[f] = base + (size_t)(2 * g->nf + f) * fb;
      if (g->ndim == 3) g->scratch[f] = base + (size_t)(3 * g->nf + f) * fb;
    }
  }
  g->staging = nullptr;
  g->shat_valid = false;
  ensure_tiles(g);
  g->step_arr = 1;   // every pass in place: T and S^ only
  ss_status st = SS_OK;
  for (int f = 0; f < g->nf && st == SS_OK; ++f) st = set_field_t<T>(g, f, fields[f]);
  if (st == SS_OK && nsteps > 0) st = ensure_shat<T>(g);
  for (int64_t i = 0; i < nsteps && st == SS_OK; ++i) st = step_once<T>(g, nullptr);
  for (int f = 0; f < g->nf && st == SS_OK; ++f) st = get_field_t<T>(g, f, fields[f]);
  for (int f = 0; f < 2; ++f) {
    g->state[f] = keep_state[f];
    g->scratch[f] = keep_scratch[f];
    g->shat[f] = keep_shat[f];
    g->scratch2[f] = keep_scratch2[f];
  }
  g->staging = keep_staging;
  g->shat_valid = keep_valid;
  g->step_arr = keep_arr;
  return st;
}

}  // namespace

extern "C" {

ss_status ss_noalloc_scratch_bytes(ss_grid g, size_t* need, size_t* limit) {
  if (!g || !need || !limit) return fail(SS_ERR_ARG, "ss_noalloc_scratch_bytes: null argument");
  if (!g->has_model) return fail(SS_ERR_STATE, "ss_noalloc_scratch_bytes: call ss_set_model first");
  *need = noalloc_arrays(g) * align_up(g->field_bytes());
  *limit = (size_t)SS_NOALLOC_SCRATCH_BYTES;
  return SS_OK;
}

ss_status ss_step_fields_noalloc(ss_grid g, void* const fields[], int64_t nsteps) {
  if (!g || !fields) return fail(SS_ERR_ARG, "ss_step_fields_noalloc: null argument");
  if (nsteps < 0) return fail(SS_ERR_ARG, "ss_step_fields_noalloc: nsteps must be >= 0");
  if (!g->has_model) return fail(SS_ERR_STATE, "ss_step_fields_noalloc: call ss_set_model first");
  if (g->solver == 1) return fail(SS_ERR_UNSUPPORTED, "ss_step_fields_noalloc: spectral solver only");
  for (int f = 0; f < g->nf; ++f)
    if (!fields[f]) return fail(SS_ERR_ARG, "ss_step_fields_noalloc: field %d is null", f);
  const size_t need = noalloc_arrays(g) * align_up(g->field_bytes());
  if (need > (size_t)SS_NOALLOC_SCRATCH_BYTES)
    return fail(SS_ERR_ARG, "ss_step_fields_noalloc: this grid needs %zu bytes of scratch, the library's fixed array holds %zu",
                need, (size_t)SS_NOALLOC_SCRATCH_BYTES);
  if (g->stream) {   // the null stream is the current device's
    int sdev = -1, cdev = -1;
    SS_TRY(hip_check(hipStreamGetDevice(g->stream, &sdev), "ss_step_fields_noalloc: stream device"));
    SS_TRY(hip_check(hipGetDevice(&cdev), "ss_step_fields_noalloc: current device"));
    if (sdev != cdev)
      return fail(SS_ERR_ARG, "ss_step_fields_noalloc: the grid's stream is on device %d, device %d is current", sdev, cdev);
  }
  void* base = nullptr;
  SS_TRY(scratch_for_current_device(&base));
  return g->dtype == SS_F64 ? step_fields_t<double>(g, fields, nsteps, (char*)base)
                            : step_fields_t<float>(g, fields, nsteps, (char*)base);
}

ss_status ss_check_finite(ss_grid g, int* nonfinite_fields) {
  if (!g || !nonfinite_fields) return fail(SS_ERR_ARG, "ss_check_finite: null argument");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_check_finite: model and workspace must be set first");
  for (int f = 0; f < g->nf; ++f)
    if (!g->field_set[f]) return fail(SS_ERR_STATE, "ss_check_finite: field %d was never set", f);
  ss::FiniteArgs a;
  memset(&a, 0, sizeof(a));
  for (int f = 0; f < g->nf; ++f) a.arr[f] = g->state[f];
  a.narr = g->nf;
  a.n = g->cells();
  a.flag = (unsigned*)g->staging;
  SS_TRY(hip_check(g->dtype == SS_F64 ? ss::run_finite<double>(a, g->stream) : ss::run_finite<float>(a, g->stream),
                   "ss_check_finite: launch"));
  unsigned flag[2] = {0u, 0u};
  SS_TRY(hip_check(hipMemcpyAsync(flag, g->staging, sizeof(flag), hipMemcpyDeviceToHost, g->stream),
                   "ss_check_finite: copy"));
  SS_TRY(hip_check(hipStreamSynchronize(g->stream), "ss_check_finite: synchronise"));
  int mask = 0;
  for (int f = 0; f < g->nf; ++f)
    if (flag[f]) mask |= 1 << f;
  *nonfinite_fields = mask;
  if (mask) return fail(SS_ERR_NONFINITE, "ss_check_finite: non-finite values in field mask %d", mask);
  return SS_OK;
}

ss_status ss_structure_factor_nbins(ss_grid g, int* nbins) {
  if (!g || !nbins) return fail(SS_ERR_ARG, "ss_structure_factor_nbins: null argument");
  *nbins = sf_nbins(g);
  return SS_OK;
}

ss_status ss_structure_factor(ss_grid g, int field, double* s_out, int64_t* n_out, int nbins) {
  if (!g || !s_out || !n_out) return fail(SS_ERR_ARG, "ss_structure_factor: null argument");
  if (g->solver == 1) return fail(SS_ERR_UNSUPPORTED, "ss_structure_factor: spectral solver only");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_structure_factor: model and workspace must be set first");
  if (field < 0 || field >= g->nf) return fail(SS_ERR_ARG, "ss_structure_factor: field %d out of range", field);
  if (!g->field_set[field]) return fail(SS_ERR_STATE, "ss_structure_factor: field %d was never set", field);
  if (nbins != sf_nbins(g))
    return fail(SS_ERR_ARG, "ss_structure_factor: nbins must be %d for this grid", sf_nbins(g));
  if (!sf_isotropic(g))
    return fail(SS_ERR_UNSUPPORTED, "ss_structure_factor: the box must have the same length along every axis");
  return g->dtype == SS_F64 ? sf_run<double>(g, field, s_out, n_out, nbins)
                            : sf_run<float>(g, field, s_out, n_out, nbins);
}

ss_status ss_step_n_profiled(ss_grid g, int64_t nsteps, double* pass_ms, int64_t* pass_count,
                             int npass) {
  if (!g) return fail(SS_ERR_ARG, "ss_step_n_profiled: null grid");
  if (g->solver == 1) return fail(SS_ERR_UNSUPPORTED, "ss_step_n_profiled: spectral solver only");
  if (!pass_ms || !pass_count || npass <= 0) return fail(SS_ERR_ARG, "ss_step_n_profiled: null outputs");
  if (nsteps < 0) return fail(SS_ERR_ARG, "ss_step_n_profiled: nsteps must be >= 0");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_step_n_profiled: model and workspace must be set first");
  for (int f = 0; f < g->nf; ++f)
    if (!g->field_set[f]) return fail(SS_ERR_STATE, "ss_step_n_profiled: field %d was never set", f);
  const int per_step = g->ndim == 2 ? 2 : 2 * g->nf + 2;
  if (nsteps * per_step > PassTimer::kMaxLaunches)
    return fail(SS_ERR_ARG, "ss_step_n_profiled: at most %d steps per call",
                (int)(PassTimer::kMaxLaunches / per_step));
  PassTimer* pt = new (std::nothrow) PassTimer();
  if (!pt) return fail(SS_ERR_ARG, "ss_step_n_profiled: out of host memory");
  const int nev = (int)(2 * nsteps * per_step);
  ss_status st = SS_OK;
  int created = 0;
  for (; created < nev; ++created) {
    st = hip_check(hipEventCreate(&pt->ev[created]), "hipEventCreate");
    if (st != SS_OK) break;
  }
  if (st == SS_OK && nsteps > 0) st = g->dtype == SS_F64 ? ensure_shat<double>(g) : ensure_shat<float>(g);
  for (int64_t i = 0; st == SS_OK && i < nsteps; ++i)
    st = g->dtype == SS_F64 ? step_once<double>(g, pt) : step_once<float>(g, pt);
  if (st == SS_OK) st = hip_check(hipStreamSynchronize(g->stream), "ss_step_n_profiled: synchronise");
  if (st == SS_OK) {
    for (int i = 0; i < npass; ++i) {
      pass_ms[i] = 0.0;
      pass_count[i] = 0;
    }
    for (int u = 0; u < pt->used; ++u) {
      float ms = 0.f;
      st = hip_check(hipEventElapsedTime(&ms, pt->ev[2 * u], pt->ev[2 * u + 1]), "hipEventElapsedTime");
      if (st != SS_OK) break;
      const int k = pt->kind[u];
      if (k >= 0 && k < npass) {
        pass_ms[k] += ms;
        pass_count[k] += 1;
      }
    }
  }
  for (int e = 0; e < created; ++e) hipEventDestroy(pt->ev[e]);
  delete pt;
  return st;
}

ss_status ss_time_pass(ss_grid g, int pass, int nlaunch, double* mean_ms) {
  if (g && g->solver == 1) return fail(SS_ERR_UNSUPPORTED, "ss_time_pass: spectral solver only");
  if (!g || !mean_ms) return fail(SS_ERR_ARG, "ss_time_pass: null argument");
  if (nlaunch < 1 || nlaunch > 100000) return fail(SS_ERR_ARG, "ss_time_pass: nlaunch must be in [1, 100000]");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_time_pass: model and workspace must be set first");
  ensure_tiles(g);
  hipEvent_t e0, e1;
  SS_TRY(hip_check(hipEventCreate(&e0), "hipEventCreate"));
  ss_status st = hip_check(hipEventCreate(&e1), "hipEventCreate");
  if (st != SS_OK) {
    hipEventDestroy(e0);
    return st;
  }
  auto one = [&]() {
    return g->dtype == SS_F64 ? launch_timed_pass<double>(g, pass, ss::LaunchEvents())
                              : launch_timed_pass<float>(g, pass, ss::LaunchEvents());
  };
  st = one();  // warm-up
  if (st == SS_OK) st = hip_check(hipEventRecord(e0, g->stream), "hipEventRecord");
  for (int i = 0; st == SS_OK && i < nlaunch; ++i) st = one();
  if (st == SS_OK) st = hip_check(hipEventRecord(e1, g->stream), "hipEventRecord");
  if (st == SS_OK) st = hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
  float ms = 0.f;
  if (st == SS_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  if (st == SS_OK) *mean_ms = (double)ms / nlaunch;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return st;
}

ss_status ss_autotune(ss_grid g, int reps) {
  if (g && g->solver == 1) return fail(SS_ERR_UNSUPPORTED, "ss_autotune: spectral solver only");
  if (!g) return fail(SS_ERR_ARG, "ss_autotune: null grid");
  if (reps < 1 || reps > 1000) return fail(SS_ERR_ARG, "ss_autotune: reps must be in [1, 1000]");
  if (!g->has_model || !g->ws) return fail(SS_ERR_STATE, "ss_autotune: model and workspace must be set first");
  ensure_tiles(g);
  return g->dtype == SS_F64 ? autotune_t<double>(g, reps) : autotune_t<float>(g, reps);
}

ss_status ss_get_tiles(ss_grid g, int tiles[6]) {
  if (!g || !tiles) return fail(SS_ERR_ARG, "ss_get_tiles: null argument");
  if (!g->has_model) return fail(SS_ERR_STATE, "ss_get_tiles: call ss_set_model first");
  ensure_tiles(g);
  tiles[0] = g->tile_x_step;
  tiles[1] = g->tile_k;
  tiles[2] = g->tile_y;
  tiles[3] = g->tile_x_io;
  tiles[4] = g->tile_x_ppb;
  tiles[5] = 1 << g->lb;
  return SS_OK;
}

ss_status ss_set_tiles(ss_grid g, const int tiles[6]) {
  if (!g || !tiles) return fail(SS_ERR_ARG, "ss_set_tiles: null argument");
  if (!g->has_model) return fail(SS_ERR_STATE, "ss_set_tiles: call ss_set_model first");
  const int esz = esz_of(g);
  const int64_t rows = g->n[1] * g->n[2];
  if (tiles[0] && !ss::x_tile_ok(esz, (int)g->n[0], g->nf, rows, tiles[0]))
    return fail(SS_ERR_ARG, "ss_set_tiles: x tile %d not valid for this grid", tiles[0]);
  if (tiles[1] && !ss::k_tile_ok(esz, nlast(g), nlines_k(g), g->ndim == 3, tiles[1]))
    return fail(SS_ERR_ARG, "ss_set_tiles: k tile %d not valid for this grid", tiles[1]);
  if (g->ndim == 3 && tiles[2] && !ss::y_tile_ok(esz, (int)g->n[1], g->n[2], tiles[2]))
    return fail(SS_ERR_ARG, "ss_set_tiles: y tile %d not valid for this grid", tiles[2]);
  if (tiles[3] && !ss::x_tile_ok(esz, (int)g->n[0], 1, rows, tiles[3]))
    return fail(SS_ERR_ARG, "ss_set_tiles: x io tile %d not valid for this grid", tiles[3]);
  if (tiles[4] < 0 || tiles[4] > 64) return fail(SS_ERR_ARG, "ss_set_tiles: tiles per block must be in [0, 64]");
  ensure_tiles(g);
  if (tiles[5] && !blk_ok(g, tiles[5])) return fail(SS_ERR_ARG, "ss_set_tiles: row block %d not valid for this grid", tiles[5]);
  if (tiles[5] && ilog2i(tiles[5]) != g->lb && (g->field_set[0] || g->field_set[1]))
    return fail(SS_ERR_STATE, "ss_set_tiles: the row block can change only before any field is set");
  if (tiles[4] > 1) {
    const int r = tiles[0] ? tiles[0] : ss::x_tile_default(esz, (int)g->n[0], g->nf, rows);
    if (!ss::x_pp_ok(esz, (int)g->n[0], g->nf, rows, r))
      return fail(SS_ERR_ARG, "ss_set_tiles: x tile %d cannot run persistent", r);
  }
  g->tile_x_step = tiles[0];
  g->tile_k = tiles[1];
  g->tile_y = g->ndim == 3 ? tiles[2] : 0;
  g->tile_x_io = tiles[3];
  g->tile_x_ppb = tiles[4];
  if (tiles[5]) g->lb = ilog2i(tiles[5]);
  ensure_tiles(g);
  return SS_OK;
}

ss_status ss_bind_mass_log(ss_grid g, double* device_ptr, int64_t capacity) {
  if (!g) return fail(SS_ERR_ARG, "ss_bind_mass_log: null grid");
  if (device_ptr && capacity < 0) return fail(SS_ERR_ARG, "ss_bind_mass_log: negative capacity");
  g->mass_log = device_ptr;
  g->log_cap = device_ptr ? capacity : 0;
  g->log_count = 0;
  return SS_OK;
}

ss_status ss_mass_log_count(ss_grid g, int64_t* count) {
  if (!g || !count) return fail(SS_ERR_ARG, "ss_mass_log_count: null argument");
  *count = g->log_count;
  return SS_OK;
}

ss_status ss_mass_log(ss_grid g, double* dst_host, int64_t max, int64_t* rows) {
  if (rows) *rows = 0;
  if (!g) return fail(SS_ERR_ARG, "ss_mass_log: null grid");
  if (max < 0) return fail(SS_ERR_ARG, "ss_mass_log: negative max");
  if (!dst_host && max > 0) return fail(SS_ERR_ARG, "ss_mass_log: null destination");
  if (!g->mass_log) return fail(SS_ERR_STATE, "ss_mass_log: no mass log is bound");
  const int64_t n = std::min(max, std::min(g->log_count, g->log_cap));
  SS_TRY(hip_check(hipStreamSynchronize(g->stream), "ss_mass_log: synchronise"));
  if (n > 0)
    SS_TRY(hip_check(hipMemcpy(dst_host, g->mass_log, sizeof(double) * (size_t)n * (size_t)g->nf,
                               hipMemcpyDeviceToHost), "ss_mass_log: copy"));
  if (rows) *rows = n;
  return SS_OK;
}

ss_status ss_set_stream(ss_grid g, void* stream) {
  if (!g) return fail(SS_ERR_ARG, "ss_set_stream: null grid");
  g->stream = (hipStream_t)stream;
  return SS_OK;
}

ss_status ss_batch_create(const ss_grid* grids, int count, ss_batch* out) {
  if (!out) return fail(SS_ERR_ARG, "ss_batch_create: out is null");
  *out = nullptr;
  if (!grids || count < 1 || count > 65536) return fail(SS_ERR_ARG, "ss_batch_create: need 1..65536 grids");
  for (int i = 0; i < count; ++i) {
    ss_grid g = grids[i];
    if (!g) return fail(SS_ERR_ARG, "ss_batch_create: grid %d is null", i);
    if (g->ndim != 2) return fail(SS_ERR_UNSUPPORTED, "ss_batch_create: grid %d is not 2D", i);
    if (!g->has_model) return fail(SS_ERR_STATE, "ss_batch_create: grid %d has no model", i);
    if (g->solver != 0) return fail(SS_ERR_UNSUPPORTED, "ss_batch_create: grid %d uses the finite-difference solver", i);
    if (g->nf != 1) return fail(SS_ERR_UNSUPPORTED, "ss_batch_create: grid %d has a two-field model", i);
    if (g->nlm != ss::NLIN_POLY || g->scheme != 0)
      return fail(SS_ERR_UNSUPPORTED, "ss_batch_create: grid %d: batches take the fixed one-field models", i);
    if (!g->ws) return fail(SS_ERR_STATE, "ss_batch_create: grid %d has no workspace", i);
    if (!batch_size_ok(g->n[0]) || !batch_size_ok(g->n[1]))
      return fail(SS_ERR_UNSUPPORTED, "ss_batch_create: grid %d size outside [64, 2048]", i);
    if (g->dtype != grids[0]->dtype) return fail(SS_ERR_ARG, "ss_batch_create: mixed dtypes");
    if (g->stream != grids[0]->stream) return fail(SS_ERR_ARG, "ss_batch_create: mixed streams");
  }
  // Members step in parallel within a launch: none may share state with
  // another (a grid listed twice, or two grids bound to overlapping
  // workspaces, would be written by two work items at once).
  {
    std::vector<std::pair<uintptr_t, uintptr_t>> used((size_t)count);
    for (int i = 0; i < count; ++i) {
      size_t need = 0;
      SS_TRY(ss_workspace_size(grids[i], &need));
      used[(size_t)i] = {(uintptr_t)grids[i]->ws, (uintptr_t)grids[i]->ws + need};
    }
    std::sort(used.begin(), used.end());
    for (size_t i = 1; i < used.size(); ++i)
      if (used[i].first < used[i - 1].second)
        return fail(SS_ERR_ARG, "ss_batch_create: two members share workspace memory (a grid listed twice?)");
  }
  ss_batch b = new (std::nothrow) ss_batch_s();
  if (!b) return fail(SS_ERR_ARG, "ss_batch_create: out of host memory");
  b->grids.assign(grids, grids + count);
  b->dtype = grids[0]->dtype;
  b->stream = grids[0]->stream;
  for (int i = 0; i < count; ++i) b->order.push_back(i);
  // largest members first: their tiles start early, the small ones fill the tail
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int a, int c) { return b->grids[a]->cells() > b->grids[c]->cells(); });
  *out = b;
  return SS_OK;
}

ss_status ss_batch_workspace_size(ss_batch b, size_t* bytes) {
  if (!b || !bytes) return fail(SS_ERR_ARG, "ss_batch_workspace_size: null argument");
  *bytes = 2 * batch_table_bytes(b) + batch_sync_bytes(b);
  return SS_OK;
}

ss_status ss_batch_bind_workspace(ss_batch b, void* device_ptr, size_t bytes) {
  if (!b || !device_ptr) return fail(SS_ERR_ARG, "ss_batch_bind_workspace: null argument");
  if (((uintptr_t)device_ptr) % kAlign) return fail(SS_ERR_ARG, "ss_batch_bind_workspace: pointer not 256-byte aligned");
  if (bytes < 2 * batch_table_bytes(b) + batch_sync_bytes(b))
    return fail(SS_ERR_ARG, "ss_batch_bind_workspace: workspace too small");
  b->ws = device_ptr;
  b->ws_bytes = bytes;
  b->uploaded = false;
  // the counters and the error flag start at zero: ss_batch_check reads the
  // flag whatever form ran (the single launches reset it as they start)
  return hip_check(hipMemsetAsync((char*)device_ptr + 2 * batch_table_bytes(b), 0, batch_sync_bytes(b), b->stream),
                   "ss_batch_bind_workspace: clear the counters");
}

ss_status ss_batch_autotune(ss_batch b, int reps) {
  if (!b) return fail(SS_ERR_ARG, "ss_batch_autotune: null batch");
  if (reps < 1 || reps > 1000) return fail(SS_ERR_ARG, "ss_batch_autotune: reps must be in [1, 1000]");
  if (!b->ws) return fail(SS_ERR_STATE, "ss_batch_autotune: bind the batch workspace first");
  int best_t = 0;
  float best = 1e30f;
  for (int threads : {128, 256, 512}) {
    std::vector<ss::BatchMember> t1, t2;
    int xt, kt, tx;
    uint32_t lx, lk;
    if (!build_batch_table(b, threads, t1, t2, xt, kt, lx, lk, tx)) continue;
    SS_TRY(batch_upload(b, threads));
    auto launch = [&](ss::LaunchEvents ev) {
      // x launch and k launch (on the tuning table) timed together
      ss::LaunchEvents ex, ek;
      ex.start = ev.start;
      ek.stop = ev.stop;
      return b->dtype == SS_F64 ? batch_launch_step<double>(b, true, ex, ek)
                                : batch_launch_step<float>(b, true, ex, ek);
    };
    float ms;
    SS_TRY(time_launch(b->grids[0], launch, reps, &ms));
    if (ms < best) {
      best = ms;
      best_t = threads;
    }
  }
  if (!best_t) return fail(SS_ERR_UNSUPPORTED, "ss_batch_autotune: no block size fits every member");
  SS_TRY(batch_upload(b, best_t));
  if (!b->mode_set) {
    // grouped launches against the single launch over a run of steps
    // (on the tuning table, which leaves the fields alone)
    b->mode = 0;
    if (batch_single_ok(b)) {
      const int64_t nrun = 8;
      auto grouped = [&](ss::LaunchEvents ev) {
        for (int64_t i = 0; i < nrun; ++i) {
          ss::LaunchEvents ex, ek;
          if (i == 0) ex.start = ev.start;
          if (i == nrun - 1) ek.stop = ev.stop;
          SS_TRY(b->dtype == SS_F64 ? batch_launch_step<double>(b, true, ex, ek)
                                    : batch_launch_step<float>(b, true, ex, ek));
        }
        return SS_OK;
      };
      auto single = [&](ss::LaunchEvents ev) {
        return b->dtype == SS_F64 ? batch_launch_single<double>(b, nrun, true, ev)
                                  : batch_launch_single<float>(b, nrun, true, ev);
      };
      auto coop = [&](ss::LaunchEvents ev) {
        return b->dtype == SS_F64 ? batch_launch_coop<double>(b, nrun, true, ev)
                                  : batch_launch_coop<float>(b, nrun, true, ev);
      };
      float tg, tp, tc = 1e30f;
      SS_TRY(time_launch(b->grids[0], grouped, reps, &tg));
      SS_TRY(time_launch(b->grids[0], single, reps, &tp));
      SS_TRY(batch_check_error(b));
      // a device that refuses the cooperative launch leaves that form out
      if (time_launch(b->grids[0], coop, reps, &tc) != SS_OK) {
        (void)hipGetLastError();
        tc = 1e30f;
      }
      SS_TRY(batch_check_error(b));
      if (tp < tg && tp < tc) b->mode = 1;
      else if (tc < tg) b->mode = 2;
    }
  }
  return SS_OK;
}

ss_status ss_batch_step_n(ss_batch b, int64_t nsteps) {
  if (!b) return fail(SS_ERR_ARG, "ss_batch_step_n: null batch");
  if (nsteps < 0) return fail(SS_ERR_ARG, "ss_batch_step_n: nsteps must be >= 0");
  if (!b->ws) return fail(SS_ERR_STATE, "ss_batch_step_n: bind the batch workspace first");
  SS_TRY(batch_check_members(b));
  if (!b->uploaded) SS_TRY(batch_upload(b, b->threads));
  if (nsteps > 0) SS_TRY(batch_refresh(b));
  SS_TRY(batch_run(b, nsteps));
  for (ss_grid g : b->grids) g->log_count += nsteps;
  return SS_OK;
}

ss_status ss_batch_capture(ss_batch b, int64_t nsteps) {
  if (!b) return fail(SS_ERR_ARG, "ss_batch_capture: null batch");
  if (nsteps < 1) return fail(SS_ERR_ARG, "ss_batch_capture: nsteps must be >= 1");
  if (!b->stream) return fail(SS_ERR_ARG, "ss_batch_capture: the null stream cannot be captured");
  if (!b->ws) return fail(SS_ERR_STATE, "ss_batch_capture: bind the batch workspace first");
  SS_TRY(batch_check_members(b));
  if (!b->uploaded) SS_TRY(batch_upload(b, b->threads));
  if (b->exec) {
    hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  if (b->graph) {
    hipGraphDestroy(b->graph);
    b->graph = nullptr;
  }
  SS_TRY(batch_refresh(b));   // outside the capture
  b->coop_direct = false;
  if (b->mode == 2) {
    // the run is one launch already: ss_batch_launch issues it directly
    // (a cooperative launch is not recorded into a graph)
    if (!b->coop_blocks) SS_TRY(b->dtype == SS_F64 ? batch_coop_size<double>(b) : batch_coop_size<float>(b));
    if (nsteps > batch_coop_max_steps(b))
      return fail(SS_ERR_ARG, "ss_batch_capture: %lld steps do not fit one cooperative launch", (long long)nsteps);
    b->coop_direct = true;
    b->graph_steps = nsteps;
    return SS_OK;
  }
  SS_TRY(hip_check(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture"));
  ss_status st = batch_run(b, nsteps);
  hipGraph_t graph = nullptr;
  ss_status st2 = hip_check(hipStreamEndCapture(b->stream, &graph), "hipStreamEndCapture");
  if (st != SS_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (st2 != SS_OK) return st2;
  b->graph = graph;
  SS_TRY(hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate"));
  b->graph_steps = nsteps;
  return SS_OK;
}

ss_status ss_batch_launch(ss_batch b) {
  if (!b) return fail(SS_ERR_ARG, "ss_batch_launch: null batch");
  if (!b->exec && !b->coop_direct) return fail(SS_ERR_STATE, "ss_batch_launch: nothing captured");
  SS_TRY(batch_check_members(b));
  SS_TRY(batch_refresh(b));
  if (b->coop_direct) {
    if (b->mode != 2) return fail(SS_ERR_STATE, "ss_batch_launch: the mode changed since the capture");
    SS_TRY(batch_run(b, b->graph_steps));
  } else {
    SS_TRY(hip_check(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch"));
  }
  for (ss_grid g : b->grids) g->log_count += b->graph_steps;
  return SS_OK;
}

ss_status ss_batch_set_mode(ss_batch b, int mode) {
  if (!b) return fail(SS_ERR_ARG, "ss_batch_set_mode: null batch");
  if (mode < 0 || mode > 2) return fail(SS_ERR_ARG, "ss_batch_set_mode: mode %d is not 0, 1 or 2", mode);
  if (!b->ws) return fail(SS_ERR_STATE, "ss_batch_set_mode: bind the batch workspace first");
  if (!b->uploaded) SS_TRY(batch_upload(b, b->threads));
  if (mode != 0 && !batch_single_ok(b))
    return fail(SS_ERR_UNSUPPORTED, "ss_batch_set_mode: the single launches need one block size for both passes");
  b->mode = mode;
  b->mode_set = true;
  return SS_OK;
}

ss_status ss_batch_get_mode(ss_batch b, int* mode) {
  if (!b || !mode) return fail(SS_ERR_ARG, "ss_batch_get_mode: null argument");
  *mode = b->mode;
  return SS_OK;
}

ss_status ss_batch_set_wait_limit(ss_batch b, unsigned limit) {
  if (!b) return fail(SS_ERR_ARG, "ss_batch_set_wait_limit: null batch");
  b->spin_limit = limit;
  return SS_OK;
}

ss_status ss_batch_check(ss_batch b) {
  if (!b) return fail(SS_ERR_ARG, "ss_batch_check: null batch");
  return batch_check_error(b);
}

ss_status ss_batch_info(ss_batch b, int info[3]) {
  if (!b || !info) return fail(SS_ERR_ARG, "ss_batch_info: null argument");
  info[0] = b->threads;
  info[1] = b->x_total;
  info[2] = b->k_total;
  return SS_OK;
}

ss_status ss_batch_destroy(ss_batch b) {
  if (!b) return SS_OK;
  // a launched graph may still be running: its nodes read the batch's
  // tables and the caller's buffers
  (void)hipStreamSynchronize(b->stream);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  delete b;
  return SS_OK;
}

ss_status ss_adjoint_workspace_size(ss_grid g, int64_t nsteps, int K, size_t* bytes) {
  if (g && g->solver == 1) return fail(SS_ERR_UNSUPPORTED, "ss_adjoint_workspace_size: spectral solver only");
  if (!g || !bytes) return fail(SS_ERR_ARG, "ss_adjoint_workspace_size: null argument");
  if (!g->has_model) return fail(SS_ERR_STATE, "ss_adjoint_workspace_size: call ss_set_model first");
  if (g->model != SS_GRAY_SCOTT || g->ndim != 2)
    return fail(SS_ERR_UNSUPPORTED, "ss_adjoint_workspace_size: reverse mode is implemented for 2D Gray-Scott");
  if (g->n[0] > 1024 || g->n[1] > 1024) return fail(SS_ERR_UNSUPPORTED, "ss_adjoint_workspace_size: axes up to 1024");
  if (nsteps < 1 || K < 1) return fail(SS_ERR_ARG, "ss_adjoint_workspace_size: nsteps and K must be >= 1");
  *bytes = adj_layout(g, nsteps, K).total;
  return SS_OK;
}

ss_status ss_bind_adjoint_workspace(ss_grid g, void* device_ptr, size_t bytes, int64_t nsteps, int K) {
  if (g && g->solver == 1) return fail(SS_ERR_UNSUPPORTED, "ss_bind_adjoint_workspace: spectral solver only");
  size_t need = 0;
  SS_TRY(ss_adjoint_workspace_size(g, nsteps, K, &need));
  if (!device_ptr) return fail(SS_ERR_ARG, "ss_bind_adjoint_workspace: null pointer");
  if (((uintptr_t)device_ptr) % kAlign) return fail(SS_ERR_ARG, "ss_bind_adjoint_workspace: pointer not 256-byte aligned");
  if (bytes < need) return fail(SS_ERR_ARG, "ss_bind_adjoint_workspace: %zu bytes given, %zu needed", bytes, need);
  g->adj_ws = device_ptr;
  g->adj_bytes = bytes;
  g->adj_nsteps = nsteps;
  g->adj_K = K;
  g->adj_forward_done = false;
  return SS_OK;
}

ss_status ss_step_n_checkpointed(ss_grid g) {
  if (!g) return fail(SS_ERR_ARG, "ss_step_n_checkpointed: null grid");
  if (!g->adj_ws) return fail(SS_ERR_STATE, "ss_step_n_checkpointed: bind the adjoint workspace first");
  if (!g->ws || !g->field_set[0] || !g->field_set[1])
    return fail(SS_ERR_STATE, "ss_step_n_checkpointed: workspace and both fields must be set");
  const AdjLayout L = adj_layout(g, g->adj_nsteps, g->adj_K);
  for (int64_t i = 0; i < g->adj_nsteps; ++i) {
    if (i % g->adj_K == 0)
      for (int f = 0; f < 2; ++f)
        SS_TRY(hip_check(hipMemcpyAsync(ck_field(g, L, i / g->adj_K, f), g->state[f], g->field_bytes(),
                                        hipMemcpyDeviceToDevice, g->stream), "checkpoint copy"));
    SS_TRY(g->dtype == SS_F64 ? step_once<double>(g, nullptr, false) : step_once<float>(g, nullptr, false));
  }
  for (int i = 0; i < g->ncoef; ++i) g->adj_coef[i] = g->coef[i];
  g->adj_dt = g->dt;
  g->adj_forward_done = true;
  return SS_OK;
}

ss_status ss_adjoint_n(ss_grid g, const void* const dJ_dqT[], void* const dJ_dq0[], double* dJ_dcoef) {
  if (!g || !dJ_dqT || !dJ_dq0 || !dJ_dcoef) return fail(SS_ERR_ARG, "ss_adjoint_n: null argument");
  if (!dJ_dqT[0] || !dJ_dqT[1] || !dJ_dq0[0] || !dJ_dq0[1]) return fail(SS_ERR_ARG, "ss_adjoint_n: null field pointer");
  if (!g->adj_ws || !g->adj_forward_done)
    return fail(SS_ERR_STATE, "ss_adjoint_n: run ss_step_n_checkpointed first");
  for (int i = 0; i < g->ncoef; ++i)
    if (g->adj_coef[i] != g->coef[i]) return fail(SS_ERR_STATE, "ss_adjoint_n: coefficients changed since the forward run");
  if (g->adj_dt != g->dt) return fail(SS_ERR_STATE, "ss_adjoint_n: dt changed since the forward run");
  return g->dtype == SS_F64 ? adjoint_t<double>(g, dJ_dqT, dJ_dq0, dJ_dcoef)
                            : adjoint_t<float>(g, dJ_dqT, dJ_dq0, dJ_dcoef);
}

ss_status ss_destroy_grid(ss_grid g) {
  delete g;
  return SS_OK;
}

}  // extern "C"
