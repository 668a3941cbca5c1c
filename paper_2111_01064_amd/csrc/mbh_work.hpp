// mbh_work.hpp -- device work list and the persistent heterodyned kernel.
//
// A work list holds items (one reference and one walker batch each) and
// tiles (kBlock / G walkers of one item).  A persistent grid of workgroups
// claims tiles through one atomic counter, longest tiles first; the last
// workgroup to leave resets the counters, so a captured graph can be replayed
// without any memset.  Per-walker results depend only on the walker, its
// reference and G, never on the rest of the batch.
#pragma once

#include "mbh_kernels.hpp"

namespace mbh {

struct WorkHeader {
  int32_t n_items, n_tiles;
  int64_t total_walkers;
};

struct WorkItem {
  HetRef ref;
  const double *theta;  // [W][11]
  WalkerC *wc;          // [W] walker constants (filled by k_setup_work)
  double *lnL;          // [W]
  double *dhhh;         // [W][2] or null
  int64_t W;
  int64_t offset;       // first walker of this item in the flattened batch
  int32_t G, model;
};

struct WorkTile {
  int32_t item, G;
  int64_t w_begin;  // first walker of the tile within its item
};

// a1 for every walker of the batch (grid-stride over the flattened walkers)
static __global__ __launch_bounds__(128) void k_setup_work(const WorkHeader *__restrict__ hdr,
                                                    const WorkItem *__restrict__ items) {
  const int64_t total = hdr->total_walkers;
  const int n = hdr->n_items;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = n - 1;  // last item with offset <= t
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (items[mid].offset <= t) lo = mid;
      else hi = mid - 1;
    }
    const WorkItem &it = items[lo];
    const int64_t w = t - it.offset;
    if (w < it.W) walker_setup(it.theta + w * 11, it.model, it.ref.modes, it.wc[w]);
  }
}

template <typename R, int G, bool DH>
__device__ __forceinline__ void run_tile(const WorkItem &it, int64_t w_begin, RouteQ rq) {
  const int64_t w = w_begin + threadIdx.x / G;
  het_walker<R, G, DH>(it.ref, it.wc, w, it.W, it.lnL, it.dhhh, rq);
}

template <typename R, bool DH>
__global__ __launch_bounds__(kBlock) void k_het_work(const WorkHeader *__restrict__ hdr,
                                                     const WorkItem *__restrict__ items,
                                                     const WorkTile *__restrict__ tiles,
                                                     unsigned int *__restrict__ counters,
                                                     unsigned int *__restrict__ route_count,
                                                     int2 *__restrict__ route_list) {
  __shared__ int s_tile;
  const int n_tiles = hdr->n_tiles;
  for (;;) {
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(&counters[0], 1u);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_tile);
    __syncthreads();
    if (t >= n_tiles) break;
    const WorkTile tl = tiles[t];
    const WorkItem &it = items[tl.item];
    const RouteQ rq{route_count, route_list, tl.item};
    switch (tl.G) {
      case 1: run_tile<R, 1, DH>(it, tl.w_begin, rq); break;
      case 2: run_tile<R, 2, DH>(it, tl.w_begin, rq); break;
      case 4: run_tile<R, 4, DH>(it, tl.w_begin, rq); break;
      case 8: run_tile<R, 8, DH>(it, tl.w_begin, rq); break;
      case 16: run_tile<R, 16, DH>(it, tl.w_begin, rq); break;
      case 32: run_tile<R, 32, DH>(it, tl.w_begin, rq); break;
      default: run_tile<R, 64, DH>(it, tl.w_begin, rq); break;
    }
  }
  // every workgroup has made its last claim before it counts itself out; the
  // last one resets both counters for the next launch on this work list
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned int done = atomicAdd(&counters[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
}

// FP64 recomputation of the walkers queued by the mixed pass: one walker per
// wavefront (64 lanes), workgroups claim groups of four queue entries.
// rc[0] queue length (written by the mixed pass), rc[1] claim head, rc[2]
// workgroups done, rc[3] running total of recomputed walkers.  The last
// workgroup adds the queue length to the total and clears rc[0..2].
// A single item may be passed by value in `one` with items == nullptr.
template <bool DH>
__global__ __launch_bounds__(kBlock) void k_het_fixup(const WorkItem *__restrict__ items, WorkItem one,
                                                      const int2 *__restrict__ list, unsigned int *__restrict__ rc) {
  __shared__ int s_t;
  const unsigned int n = rc[0];
  constexpr int kPer = kBlock / 64;
  for (;;) {
    if (threadIdx.x == 0) s_t = (int)atomicAdd(&rc[1], 1u);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_t);
    __syncthreads();
    const int64_t base = (int64_t)t * kPer;
    if (base >= (int64_t)n) break;
    const int64_t idx = base + threadIdx.x / 64;
    const int2 e0 = list[idx < (int64_t)n ? idx : base];
    // one queue entry per wavefront: its fields are wave-uniform
    const int2 e = make_int2(__builtin_amdgcn_readfirstlane(e0.x), __builtin_amdgcn_readfirstlane(e0.y));
    const WorkItem &it = items ? items[e.x] : one;
    // walkers past the queue end are parked on index W (inactive)
    het_walker<double, 64, DH>(it.ref, it.wc, idx < (int64_t)n ? (int64_t)e.y : it.W, it.W, it.lnL, it.dhhh,
                               RouteQ{nullptr, nullptr, 0});
  }
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned int done = atomicAdd(&rc[2], 1u);
    if (done == gridDim.x - 1) {
      atomicAdd(&rc[3], n);
      atomicExch(&rc[0], 0u);
      atomicExch(&rc[1], 0u);
      atomicExch(&rc[2], 0u);
    }
  }
}

}  // namespace mbh
