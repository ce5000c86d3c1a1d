// Kernels of the batched step (members may differ in grid size and
// coefficients).  A device table describes the members; every tile runs
// the same size-specialised tile code the single-grid kernels run.
//
// Grouped form: one launch per pass and step covers the tiles of every
// member; block b takes tile b of the global tile numbering and finds the
// member that owns it.  One block handles one tile (a grid-stride loop
// would let the compiler hoist the per-size set-up of every size out of
// the loop and run out of registers); the hardware dispatcher balances
// the blocks, and the kernel boundary orders the passes.
//
// Single-launch form: one launch runs every step of every member.  Each
// workgroup, as it starts, draws one work item from a ticket counter in
// the order (step, x tiles of every member, k-space tiles of every member);
// per-member counters of finished tiles replace the kernel boundary: an x
// tile of step s waits until its member's k-space tiles of step s - 1 are
// done, a k-space tile until its member's x tiles of step s are.  An item
// only waits on items with smaller tickets, which workgroups that started
// earlier hold, so the launch drains whatever the number of resident
// workgroups; members advance independently, and the dispatcher keeps the
// CUs filled across step boundaries.  Every wait is bounded: when one
// runs out, an error flag is raised and every later workgroup leaves at
// once (the host reports it).
//
// Cooperative form: one launch runs every step with a fixed set of
// workgroups, all resident at once (a cooperative launch).  In each step
// workgroup g takes x tiles g, g + G, g + 2G, ... of the global numbering,
// meets every other workgroup at a device-wide barrier, takes its k-space
// tiles the same way and meets them again.  Two barriers a step replace
// the two kernel boundaries of the grouped form, with none of the
// single-launch form's per-item waits: for a few small grids, whose steps
// are otherwise mostly launch gaps.
#pragma once

#include "ss_kernels.hpp"

namespace ss {

struct BatchMember {
  XArgs x;          // x-pass arguments (rows_per_block set for the block size)
  KArgs k;          // k-space arguments (lines_per_block set)
  int nx, ny;
  int x_first, x_tiles;   // tiles [x_first, x_first + x_tiles) of the x launch
  int k_first, k_tiles;
  int xsp;          // x pass at the small grids' 4 points per thread (x_small)
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

// one x tile of a member of N-point rows, with the member's points per thread
template <typename T, int N>
__device__ __forceinline__ void batch_x_tile(const BatchMember& m, int64_t blk, C<T>* lds, int tid) {
  if constexpr (N <= 512) {
    if (m.xsp) {
      xpass_body<T, N, 1, XMODE_STEP, NLIN_POLY, false, true>(m.x, blk, lds, tid);
      return;
    }
  }
  xpass_body<T, N, 1, XMODE_STEP, NLIN_POLY>(m.x, blk, lds, tid);
}

template <typename T>
__global__ void __launch_bounds__(512) xpass_grouped(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  const int tile = blockIdx.x;
  if (tile < b.x_total) {
    const int i = batch_find(b.m, b.count, tile, false);
    const int64_t blk = tile - b.m[i].x_first;
    switch (b.m[i].nx) {
#define SS_CASE(n)                                                  \
  case n:                                                           \
    batch_x_tile<T, n>(b.m[i], blk, lds, threadIdx.x);             \
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
    kpass_body<T, n, true, 0, k_pts((int)sizeof(C<T>), n)>(a, bx, 0, lds); \
    break;
      SS_BATCH_SIZES(SS_CASE)
#undef SS_CASE
    }
  }
}

// ---- single-launch form ------------------------------------------------------
struct BatchSync {
  unsigned* ctl;      // [0] next ticket, [1] error flag (a bounded wait ran out)
  unsigned* xdone;    // per member: x tiles finished in this launch
  unsigned* kdone;    // per member: k-space tiles finished in this launch
  int nsteps;
  unsigned spin_limit;
};

template <typename T>
__global__ void __launch_bounds__(256) batch_sync_reset(BatchArgs b, BatchSync y) {
  for (int i = threadIdx.x; i < b.count; i += blockDim.x) {
    y.xdone[i] = 0u;
    y.kdone[i] = 0u;
  }
  if (threadIdx.x == 0) {
    y.ctl[0] = 0u;
    y.ctl[1] = 0u;
  }
}

// Thread 0 only: wait until *c >= target (acquire), unless the error flag
// is raised or the bounded wait runs out (which raises it).
__device__ __forceinline__ bool batch_wait(const unsigned* c, unsigned target, unsigned* ctl, unsigned limit) {
  unsigned n = 0;
  while (__hip_atomic_load(c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
    if (++n > limit) {
      __hip_atomic_store(ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return true;
}

template <typename T>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(SS_KWAVES)))
batch_single(BatchArgs b, BatchSync y) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  __shared__ unsigned s_ticket;
  __shared__ int s_go;
  const unsigned per_step = (unsigned)(b.x_total + b.k_total);
  const unsigned total = per_step * (unsigned)y.nsteps;
  // one work item per workgroup, in the order workgroups start (not their
  // index): a workgroup only waits on items that started before it
  if (threadIdx.x == 0) {
    int go = 0;
    unsigned t = total;
    if (!__hip_atomic_load(y.ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      t = atomicAdd(y.ctl, 1u);
      if (t < total) {
        const unsigned step = t / per_step, r = t - step * per_step;
        if (r < (unsigned)b.x_total) {
          const int i = batch_find(b.m, b.count, (int)r, false);
          go = batch_wait(y.kdone + i, step * (unsigned)b.m[i].k_tiles, y.ctl, y.spin_limit);
        } else {
          const int i = batch_find(b.m, b.count, (int)(r - b.x_total), true);
          go = batch_wait(y.xdone + i, (step + 1) * (unsigned)b.m[i].x_tiles, y.ctl, y.spin_limit);
        }
      }
    }
    s_ticket = t;
    s_go = go;
  }
  __syncthreads();
  if (!s_go) return;
  const unsigned t = s_ticket;
  const unsigned step = t / per_step, r = t - step * per_step;
  const bool xside = r < (unsigned)b.x_total;
  const int tile = xside ? (int)r : (int)(r - b.x_total);
  const int i = batch_find(b.m, b.count, tile, !xside);
  if (xside) {
    const int64_t blk = tile - b.m[i].x_first;
    switch (b.m[i].nx) {
#define SS_CASE(n)                                           \
  case n:                                                    \
    batch_x_tile<T, n>(b.m[i], blk, lds, threadIdx.x);      \
    break;
      SS_BATCH_SIZES(SS_CASE)
#undef SS_CASE
    }
  } else {
    const KArgs& a = b.m[i].k;
    const int bx = tile - b.m[i].k_first;
    switch (b.m[i].ny) {
#define SS_CASE(n)                         \
  case n:                                  \
    kpass_body<T, n, true, 0, k_pts((int)sizeof(C<T>), n)>(a, bx, 0, lds); \
    break;
      SS_BATCH_SIZES(SS_CASE)
#undef SS_CASE
    }
  }
  // release: every thread's stores reach device scope before the count
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(xside ? y.xdone + i : y.kdone + i, 1u);
}

// ---- cooperative form -----------------------------------------------------------
// Device-wide barrier number `target / gridDim.x` (the counter only grows):
// every thread's stores are released to device scope, thread 0 adds one
// arrival and polls (relaxed, bounded) until every workgroup has arrived,
// then acquires.  False if the wait ran out or another workgroup's did.
__device__ __forceinline__ bool coop_barrier(unsigned* ctl, unsigned target, unsigned limit, int* s_go) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(ctl, 1u);
    unsigned n = 0;
    int go = 1;
    while (__hip_atomic_load(ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(ctl + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        go = 0;
        break;
      }
      if (++n > limit) {
        __hip_atomic_store(ctl + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        go = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_go = go;
  }
  __syncthreads();
  return *s_go != 0;
}

template <typename T>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(SS_KWAVES)))
batch_coop(BatchArgs b, BatchSync y) {
  extern __shared__ __align__(16) unsigned char ss_dyn_lds[];
  C<T>* lds = reinterpret_cast<C<T>*>(ss_dyn_lds);
  __shared__ int s_go;
  const unsigned G = gridDim.x;
  unsigned arrivals = 0;
  for (int step = 0; step < y.nsteps; ++step) {
    for (int tile = (int)blockIdx.x; tile < b.x_total; tile += (int)G) {
      // a fresh copy of the thread index per tile: nothing derived from it
      // is hoisted out of the loop (each size's set-up would stay live)
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int i = batch_find(b.m, b.count, tile, false);
        const int64_t blk = tile - b.m[i].x_first;
      switch (b.m[i].nx) {
#define SS_CASE(n)                                                \
  case n:                                                         \
    batch_x_tile<T, n>(b.m[i], blk, lds, tid);                    \
    break;
        SS_BATCH_SIZES(SS_CASE)
#undef SS_CASE
      }
      __syncthreads();   // the next tile reuses the LDS
    }
    arrivals += G;
    if (!coop_barrier(y.ctl, arrivals, y.spin_limit, &s_go)) return;
    for (int tile = (int)blockIdx.x; tile < b.k_total; tile += (int)G) {
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      const int i = batch_find(b.m, b.count, tile, true);
      const KArgs& a = b.m[i].k;
      const int bx = tile - b.m[i].k_first;
      switch (b.m[i].ny) {
#define SS_CASE(n)                                  \
  case n:                                           \
    kpass_body<T, n, true, 0, k_pts((int)sizeof(C<T>), n)>(a, bx, 0, lds, tid);     \
    break;
        SS_BATCH_SIZES(SS_CASE)
#undef SS_CASE
      }
      __syncthreads();
    }
    arrivals += G;
    if (!coop_barrier(y.ctl, arrivals, y.spin_limit, &s_go)) return;
  }
}

}  // namespace ss
