// Grouped kernels of the batched step: one launch covers the tiles of
// every member simulation of a batch (members may differ in grid size
// and coefficients).  A device table describes the members; block b takes
// tile b of the global tile numbering, finds the member that owns it and
// runs the same size-specialised tile code the single-grid kernels run.
// One block handles one tile (a grid-stride loop would let the compiler
// hoist the per-size set-up of every size out of the loop and run out of
// registers); the hardware dispatcher balances the blocks.
#pragma once

#include "ss_kernels.hpp"

namespace ss {

struct BatchMember {
  XArgs x;          // x-pass arguments (rows_per_block set for the block size)
  KArgs k;          // k-space arguments (lines_per_block set)
  int nx, ny;
  int x_first, x_tiles;   // tiles [x_first, x_first + x_tiles) of the x launch
  int k_first, k_tiles;
};

struct BatchArgs {
  const BatchMember* __restrict__ m;   // read-only during the launch
  int count;
  int x_total, k_total;
};

// member owning global tile `tile` (first[] ascending): binary search
__device__ __forceinline__ int batch_find(const BatchMember* __restrict__ m, int count, int tile,
                                          bool kside) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int f = kside ? m[mid].k_first : m[mid].x_first;
    if (f <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

#define SS_BATCH_SIZES(M) M(64) M(128) M(256) M(512) M(1024) M(2048)

template <typename T>
__global__ void __launch_bounds__(512) xpass_grouped(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  const int tile = blockIdx.x;
  if (tile < b.x_total) {
    const int i = batch_find(b.m, b.count, tile, false);
    const XArgs& a = b.m[i].x;   // read from the table as used
    const int64_t blk = tile - b.m[i].x_first;
    switch (b.m[i].nx) {
#define SS_CASE(n)                                                  \
  case n:                                                           \
    xpass_body<T, n, 1, XMODE_STEP, NLIN_POLY>(a, blk, lds);        \
    break;
      SS_BATCH_SIZES(SS_CASE)
#undef SS_CASE
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(SS_KWAVES))) kpass_grouped(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  const int tile = blockIdx.x;
  if (tile < b.k_total) {
    const int i = batch_find(b.m, b.count, tile, true);
    const KArgs& a = b.m[i].k;
    const int bx = tile - b.m[i].k_first;
    switch (b.m[i].ny) {
#define SS_CASE(n)                  \
  case n:                           \
    kpass_body<T, n, true>(a, bx, 0, lds); \
    break;
      SS_BATCH_SIZES(SS_CASE)
#undef SS_CASE
    }
  }
}

}  // namespace ss
