// mbh_work.hpp -- device work list of the batched heterodyned pass.
//
// A work list holds items (one reference and one walker batch each) and
// tiles.  A tile is kWaves chunks of one item (flattened mapping, G = 0) or
// kBlock / G walkers of one item (lane-group mapping).  Tiles are grouped by
// mapping and ordered longest first within a group; each group is one grid
// of one workgroup per tile, so the kernel of a group is compiled for its
// mapping alone (a kernel that switched over mappings would be allocated the
// registers of the largest one).  Per-walker results depend only on the
// walker, its index within its item, its reference and the mapping, never on
// the rest of the batch.
#pragma once

#include "mbh_kernels.hpp"

namespace mbh {

struct WorkHeader {
  int32_t n_items, n_tiles;
  int64_t total_walkers;
};

struct WorkTile {
  int32_t item, G;
  int64_t begin;  // first chunk (G = 0) or first walker (G > 0) of the tile
};

// a1 for every walker of the batch, one workgroup per walker tile: the first
// kWalkerTile threads set the intrinsic constants, the other kWalkerTile the
// extrinsic ones, of the same walkers
static __global__ __launch_bounds__(2 * kWalkerTile) void k_setup_work(const WorkItem *__restrict__ items,
                                                                       const WalkerTile *__restrict__ wtiles) {
  const WalkerTile &tl = wtiles[blockIdx.x];
  const WorkItem &it = tl.it;
  const int64_t w = tl.w_begin + (threadIdx.x & (kWalkerTile - 1));
  const int part = threadIdx.x < kWalkerTile ? 1 : 2;
  if (w < it.W) walker_setup(it.theta + w * 11, it.model, it.ref.modes, it.wc[w], part);
}

// Occupancy: the (2,2)-only kernels need 94 VGPRs (5 wavefronts per SIMD);
// the any-mode flattened kernels ~196, i.e. 2 per SIMD, and the mixed one is
// held to 168 for 3 (80 B of spills per lane in its FP64 recomputation
// branch; 4 % faster on a 16-source higher-mode batch, while the FP64 one
// ran 1 % slower at 3, so it stays at 2).
template <typename R, bool DH, int G, bool HM>
__global__ __launch_bounds__(kBlock, (HM && G == 0 && sizeof(R) == 4) ? 3 : 2) void k_het_tiles(
    const WorkItem *__restrict__ items,
                                                         const WorkTile *__restrict__ tiles) {
  const WorkTile tl = tiles[blockIdx.x];
  // the item's fields are uniform: load them once, up front, into scalars
  WorkItem it = items[tl.item];
  it.ref = with_meta(it.ref);
  if constexpr (G == 0) {
    const int64_t c = tl.begin + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (c < flat_chunks(it.W, it.E)) het_chunk<R, DH, HM>(it, c);
  } else {
    het_walker<R, G, DH, HM>(it, tl.begin + threadIdx.x / G);
  }
}

// Tiles of per-mode items carry these in place of G: kWaves chunks of the
// edge pass or of the cross pass (which reads the edge pass's deltas: its
// group is launched after every edge-pass group).
constexpr int kPmEdgeTiles = 128;
constexpr int kPmCrossTiles = 129;
// and, for items whose cross pass takes one workgroup per one or two walkers,
// this, with `begin` the first of them
constexpr int kPmCrossWgTiles = 130;

template <bool DH, int PASS>
__global__ __launch_bounds__(kBlock, 2) void k_pm_tiles(const WorkItem *__restrict__ items,
                                                        const WorkTile *__restrict__ tiles) {
  const WorkTile tl = tiles[blockIdx.x];
  WorkItem it = items[tl.item];
  it.ref = with_meta(it.ref);
  const int64_t c = tl.begin + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if constexpr (PASS == 1) {
    if (c < flat_chunks(it.W, it.E)) pm_chunk_edges<DH>(it, c);
  } else {
    if (c < flat_chunks(it.W, it.E2)) pm_chunk_cross<DH>(it, c);
  }
}

template <bool DH>
__global__ __launch_bounds__(kBlock) void k_pm_cross_tiles(const WorkItem *__restrict__ items,
                                                           const WorkTile *__restrict__ tiles) {
  extern __shared__ double2 pm_sd[];
  const WorkTile tl = tiles[blockIdx.x];
  pm_walker_cross<DH>(items[tl.item], tl.begin, pm_sd);
}

}  // namespace mbh
