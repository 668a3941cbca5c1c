// mbh_serve.hip -- ragged multi-source batching in one graph-captured launch
// (mbh_batch_*) and a continuous-batching request server on top of the same
// work-list kernels (mbh_server_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mbh.h"
#include "mbh_internal.hpp"
#include "mbh_work.hpp"

using namespace mbh;

HetRef ref_view(const mbh_ref *r);
int lanes_lookup(const mbh_ctx *ctx, int n_bins, int n_modes, int prec);
int popcount_modes(uint32_t m);
WorkItem make_item(const mbh_ctx *ctx, const mbh_ref *r, int G);
void launch_finish(const WorkItem *items, const WorkItem &one, const WalkerTile *wtiles, int64_t n_wtiles,
                   hipStream_t st);

// walker tiles of one item (kWalkerTile walkers each), each with a copy of
// the item's fields
static void append_wtiles(std::vector<WalkerTile> &wt, int item, const WorkItem &it) {
  for (int64_t w = 0; w < it.W; w += kWalkerTile) {
    WalkerTile t{};
    t.item = item;
    t.w_begin = w;
    t.it = it;
    wt.push_back(t);
  }
}

#define HIP_TRY(x)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess) return mbh_fail(MBH_EDEVICE, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- shared helpers
static int item_lanes(const mbh_ctx *ctx, const mbh_ref *r, int prec) {
  return lanes_lookup(ctx, r->n_bins, popcount_modes(r->modes ? r->modes : 1u), prec);
}

// tiles of one item: kWaves chunks (G = 0) or kBlock / G walkers each; cost ~
// edge evaluations per lane x modes
static int64_t tiles_of(int G, int64_t W, int E) {
  if (W <= 0) return 0;
  if (G == 0) return (flat_chunks(W, E) + kWaves - 1) / kWaves;
  const int64_t wpb = kBlock / G;
  return (W + wpb - 1) / wpb;
}

// Tile cost for the longest-first order: the work per lane, plus a small term
// that puts the tiles of louder references (larger <h0|h0>) first among
// equals: on the mixed path their walkers are the likeliest to need the FP64
// recomputation, which then overlaps the rest of the pass instead of
// trailing it.
static double tile_cost(double work, const mbh_ref *r) {
  return work + 0.05 * std::log10(1.0 + std::max(0.0, r->hh0_build));
}

static void append_tiles(std::vector<WorkTile> &tiles, std::vector<double> &cost, int item, const mbh_ref *r,
                         int G, int64_t W, int cross_wg = 0) {
  const int E = r->n_bins + 1;
  const int nm = popcount_modes(r->modes ? r->modes : 1u);
  if (W <= 0) return;
  if (r->pm) {  // per-mode reference: edge-pass tiles, then cross-pass tiles
    const int64_t n1 = flat_chunks(W, r->pm_T1);
    for (int64_t c = 0; c < n1; c += kWaves) {
      tiles.push_back(WorkTile{item, kPmEdgeTiles, c});
      cost.push_back(tile_cost(1.0, r));
    }
    if (cross_wg > 0) {  // one workgroup per cross_wg walkers
      for (int64_t w = 0; w < W; w += cross_wg) {
        tiles.push_back(WorkTile{item, kPmCrossWgTiles, w});
        cost.push_back(tile_cost(1.0, r));
      }
    } else if (r->pm_T2 > 0) {
      const int64_t n2 = flat_chunks(W, r->pm_T2 + 1);
      for (int64_t c = 0; c < n2; c += kWaves) {
        tiles.push_back(WorkTile{item, kPmCrossTiles, c});
        cost.push_back(tile_cost(1.0, r));
      }
    }
    return;
  }
  if (G == 0) {
    const int64_t nc = flat_chunks(W, E);
    for (int64_t c = 0; c < nc; c += kWaves) {
      tiles.push_back(WorkTile{item, 0, c});
      cost.push_back(tile_cost((double)nm, r));
    }
    return;
  }
  const int64_t wpb = kBlock / G;
  const double c = tile_cost((double)((E + G - 1) / G) * nm, r);
  for (int64_t w = 0; w < W; w += wpb) {
    tiles.push_back(WorkTile{item, G, w});
    cost.push_back(c);
  }
}

// tiles grouped by kernel (mapping, and the (2,2)-only or any-mode
// template), longest first within a group (stable), and the group ranges
// (G, hm, first tile, count)
struct TileGroup {
  int G, hm, prec;
  int64_t begin, count;
  size_t lds = 0;  // dynamic LDS of the group's kernel (per-walker cross pass: its largest item's deltas)
};

// The tiles arrive as runs (consecutive tiles of one item and one kernel,
// equal cost): the runs are stably sorted, which orders the tiles exactly as
// a stable sort of the tiles themselves would, at the cost of sorting the
// runs only.
static std::vector<TileGroup> order_tiles(std::vector<WorkTile> &tiles, const std::vector<double> &cost,
                                          const WorkItem *items) {
  struct Run {
    int64_t begin, count;
  };
  std::vector<Run> runs;
  for (size_t i = 0; i < tiles.size(); ++i) {
    if (i == 0 || tiles[i].item != tiles[i - 1].item || tiles[i].G != tiles[i - 1].G || cost[i] != cost[i - 1])
      runs.push_back(Run{(int64_t)i, 0});
    runs.back().count += 1;
  }
  auto hm = [&](const Run &r) { return items[tiles[r.begin].item].hm; };
  auto pr = [&](const Run &r) { return items[tiles[r.begin].item].prec; };
  std::stable_sort(runs.begin(), runs.end(), [&](const Run &a, const Run &b) {
    const WorkTile &ta = tiles[a.begin], &tb = tiles[b.begin];
    if (pr(a) != pr(b)) return pr(a) > pr(b);  // mixed-precision groups first
    if (ta.G != tb.G) return ta.G < tb.G;
    if (hm(a) != hm(b)) return hm(a) < hm(b);
    return cost[a.begin] > cost[b.begin];
  });
  std::vector<WorkTile> out;
  out.reserve(tiles.size());
  for (const Run &r : runs) out.insert(out.end(), tiles.begin() + r.begin, tiles.begin() + r.begin + r.count);
  tiles.swap(out);
  std::vector<TileGroup> groups;
  for (size_t i = 0; i < tiles.size(); ++i) {
    const int h = items[tiles[i].item].hm, p = items[tiles[i].item].prec;
    if (groups.empty() || groups.back().G != tiles[i].G || groups.back().hm != h || groups.back().prec != p)
      groups.push_back(TileGroup{tiles[i].G, h, p, (int64_t)i, 0});
    groups.back().count += 1;
    if (tiles[i].G == kPmCrossWgTiles)
      groups.back().lds = std::max(groups.back().lds, (size_t)items[tiles[i].item].pm.cross_wg *
                                                          items[tiles[i].item].pm.T1 * 3 * sizeof(double2));
  }
  return groups;
}

// Workgroups are dealt to the eight XCDs in turn (workgroup b on XCD b mod 8)
// and each XCD has its own L2.  Place the setup and main-pass work of a
// walker on one XCD, so that the main pass finds the walker constants the
// setup kernel has just written in its own L2: walker tile j of item i gets
// colour (i + j) mod 8 (so that the tiles of one temperature rung, which
// carry similar work, spread over all XCDs), the walker-tile array deals
// colours in turn, and the flattened main-pass tiles, kept in their order
// within each XCD, are dealt to the XCD of their first walker's setup tile.
// The tiles of both passes of a per-mode item follow the same rule, so that
// a walker's cross-pass tiles share one L2 and read its deltas from HBM once.
// Results do not depend on the order (each walker's partial slots are fixed).
// Dealing: position p takes the next element of colour p mod 8, or of the
// next colour (cyclically) that still has elements; the colour classes are
// formed by a counting sort.
constexpr int kXcds = 8;
template <typename T>
static void deal_by_colour(const std::vector<T> &in, const std::vector<uint8_t> &colour, T *out,
                           std::vector<int64_t> *out_colour_of_in = nullptr) {
  const int64_t n = (int64_t)in.size();
  int64_t cnt[kXcds] = {0}, head[kXcds], end[kXcds];
  for (int64_t k = 0; k < n; ++k) cnt[colour[k]] += 1;
  std::vector<int64_t> order((size_t)n);
  int64_t off = 0;
  for (int c = 0; c < kXcds; ++c) {
    head[c] = off;
    off += cnt[c];
    end[c] = off;
  }
  {
    int64_t fill[kXcds];
    for (int c = 0; c < kXcds; ++c) fill[c] = head[c];
    for (int64_t k = 0; k < n; ++k) order[(size_t)fill[colour[k]]++] = k;
  }
  for (int64_t pos = 0; pos < n; ++pos) {
    int c = (int)(pos % kXcds);
    while (head[c] == end[c]) c = (c + 1) % kXcds;
    const int64_t k = order[(size_t)head[c]++];
    out[pos] = in[(size_t)k];
    if (out_colour_of_in) (*out_colour_of_in)[(size_t)k] = pos % kXcds;
  }
}

static void xcd_align(std::vector<WorkTile> &tiles, const std::vector<TileGroup> &groups,
                      std::vector<WalkerTile> &wtiles, const WorkItem *items, int n_items) {
  std::vector<int64_t> wt_first(n_items + 1, 0);
  for (int i = 0; i < n_items; ++i) wt_first[i + 1] = wt_first[i] + (items[i].W + kWalkerTile - 1) / kWalkerTile;
  std::vector<uint8_t> colour(wtiles.size());
  for (size_t k = 0; k < wtiles.size(); ++k) {
    const int i = wtiles[k].item;
    colour[k] = (uint8_t)((i + ((int64_t)k - wt_first[i])) % kXcds);
  }
  std::vector<WalkerTile> wt2(wtiles.size());
  std::vector<int64_t> xcd_of(wtiles.size());
  deal_by_colour(wtiles, colour, wt2.data(), &xcd_of);
  wtiles.swap(wt2);
  for (const auto &g : groups) {
    if (g.G != 0 && g.G != kPmEdgeTiles && g.G != kPmCrossTiles && g.G != kPmCrossWgTiles) continue;
    std::vector<WorkTile> in(tiles.begin() + g.begin, tiles.begin() + g.begin + g.count);
    std::vector<uint8_t> col((size_t)g.count);
    for (int64_t i = 0; i < g.count; ++i) {
      const WorkTile &t = in[(size_t)i];
      // the tile's first walker: tasks per walker E (flattened main pass, per-mode edge pass) or E2
      // (per-mode chunked cross pass); the per-walker cross pass names its walker
      const int64_t w = g.G == kPmCrossWgTiles
                            ? t.begin
                            : (t.begin * kChunk) / (g.G == kPmCrossTiles ? items[t.item].E2 : items[t.item].E);
      col[(size_t)i] = (uint8_t)xcd_of[(size_t)(wt_first[t.item] + w / kWalkerTile)];
    }
    deal_by_colour(in, col, tiles.data() + g.begin);
  }
}

template <typename R, bool DH, bool HM>
static void launch_group_t(const TileGroup &g, const WorkItem *items, const WorkTile *tiles, hipStream_t st) {
  const dim3 grid((unsigned)g.count), blk(kBlock);
  const WorkTile *t = tiles + g.begin;
  switch (g.G) {
    case 0: hipLaunchKernelGGL((k_het_tiles<R, DH, 0, HM>), grid, blk, 0, st, items, t); break;
    case 1: hipLaunchKernelGGL((k_het_tiles<R, DH, 1, HM>), grid, blk, 0, st, items, t); break;
    case 2: hipLaunchKernelGGL((k_het_tiles<R, DH, 2, HM>), grid, blk, 0, st, items, t); break;
    case 4: hipLaunchKernelGGL((k_het_tiles<R, DH, 4, HM>), grid, blk, 0, st, items, t); break;
    case 8: hipLaunchKernelGGL((k_het_tiles<R, DH, 8, HM>), grid, blk, 0, st, items, t); break;
    case 16: hipLaunchKernelGGL((k_het_tiles<R, DH, 16, HM>), grid, blk, 0, st, items, t); break;
    case 32: hipLaunchKernelGGL((k_het_tiles<R, DH, 32, HM>), grid, blk, 0, st, items, t); break;
    default: hipLaunchKernelGGL((k_het_tiles<R, DH, 64, HM>), grid, blk, 0, st, items, t); break;
  }
}

template <typename R, bool DH>
static void launch_group(const TileGroup &g, const WorkItem *items, const WorkTile *tiles, hipStream_t st) {
  if (g.G == kPmEdgeTiles || g.G == kPmCrossTiles || g.G == kPmCrossWgTiles) {  // per-mode items (FP64 only)
    const dim3 grid((unsigned)g.count), blk(kBlock);
    const WorkTile *t = tiles + g.begin;
    if (g.G == kPmEdgeTiles) hipLaunchKernelGGL((k_pm_tiles<DH, 1>), grid, blk, 0, st, items, t);
    else if (g.G == kPmCrossTiles) hipLaunchKernelGGL((k_pm_tiles<DH, 2>), grid, blk, 0, st, items, t);
    else hipLaunchKernelGGL((k_pm_cross_tiles<DH>), grid, blk, g.lds, st, items, t);
    return;
  }
  if (g.hm) launch_group_t<R, DH, true>(g, items, tiles, st);
  else launch_group_t<R, DH, false>(g, items, tiles, st);
}

// setup (a1), one grid per group of tiles (main pass in the group's
// precision, with the mixed path's FP64 recomputation inside), and the
// per-walker totals; the stage mask selects 1 setup, 2 main pass, 4 totals
static void launch_work(bool dh, int64_t n_wtiles, const std::vector<TileGroup> &groups, const WalkerTile *wtiles,
                        const WorkItem *items, const WorkTile *tiles, hipStream_t st, int stages = 7) {
  if (n_wtiles <= 0) return;  // no walkers: no walker tile to read
  const dim3 nw((unsigned)n_wtiles);
  if (stages & 1) hipLaunchKernelGGL(k_setup_work, nw, dim3(2 * kWalkerTile), 0, st, items, wtiles);
  for (const TileGroup &g : groups) {
    if (!(stages & 2)) break;
    if (g.prec == MBH_FP64) {
      if (dh) launch_group<double, true>(g, items, tiles, st);
      else launch_group<double, false>(g, items, tiles, st);
    } else {
      if (dh) launch_group<float, true>(g, items, tiles, st);
      else launch_group<float, false>(g, items, tiles, st);
    }
  }
  if (!(stages & 4)) return;
  WorkItem none;
  std::memset(&none, 0, sizeof(none));
  launch_finish(items, none, wtiles, n_wtiles, st);
}

// ---------------------------------------------------------------- batch
struct mbh_batch {
  mbh_ctx *ctx = nullptr;
  CtxHold hold;
  bool dh = false;
  WorkItem *items = nullptr;
  WorkTile *tiles = nullptr;
  WalkerTile *wtiles = nullptr;
  int64_t n_wtiles = 0;
  unsigned long long *redo = nullptr;  // segments recomputed in FP64 (mixed), all launches
  std::vector<std::pair<void *, size_t>> allocs;
  std::vector<TileGroup> groups;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_free(mbh_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (auto &a : b->allocs) ctx_free(b->ctx, a.first, a.second);
  delete b;
}

template <typename T>
static mbh_status batch_alloc(mbh_batch *b, T **p, size_t n) {
  const size_t bytes = std::max<size_t>(1, n) * sizeof(T);
  mbh_status s = ctx_alloc(b->ctx, (void **)p, bytes);
  if (s == MBH_OK) b->allocs.emplace_back((void *)*p, bytes);
  return s;
}

extern "C" mbh_status mbh_batch_create_prec(mbh_ctx *ctx, int n, const mbh_ref *const *refs,
                                            const double *const *theta_dev, const int64_t *W,
                                            double *const *lnL_dev, double *const *dh_hh_dev,
                                            const mbh_precision *precs, mbh_batch **out) {
  if (!ctx || !refs || !theta_dev || !W || !lnL_dev || !out || !precs || n < 1)
    return mbh_fail(MBH_EINVAL, "bad argument");
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (precs[i] != MBH_FP64 && precs[i] != MBH_MIXED) return mbh_fail(MBH_EINVAL, "item %d: bad precision", i);
  int64_t total = 0;
  bool dh = false;
  int Kmax = 1;
  size_t pm_cells = 0;  // per-mode items: deltas at the edges, W T1 C of them
  for (int i = 0; i < n; ++i) {
    if (!refs[i] || W[i] < 0 || (W[i] > 0 && (!theta_dev[i] || !lnL_dev[i])))
      return mbh_fail(MBH_EINVAL, "item %d: null reference or buffers", i);
    if (refs[i]->ctx != ctx) return mbh_fail(MBH_EINVAL, "item %d: reference of another context", i);
    if (refs[i]->pm && precs[i] != MBH_FP64)
      return mbh_fail(MBH_EINVAL, "item %d: per-mode references are evaluated in MBH_FP64", i);
    total += W[i];
    if (dh_hh_dev && dh_hh_dev[i]) dh = true;
    Kmax = std::max(Kmax, refs[i]->pm ? flat_slots(refs[i]->pm_T1) + flat_slots(refs[i]->pm_T2 + 1)
                                      : flat_slots(refs[i]->n_bins + 1));
    if (refs[i]->pm) pm_cells += (size_t)W[i] * refs[i]->pm_T1 * 3;
  }
  if (total == 0) return mbh_fail(MBH_EINVAL, "batch of %d items holds no walkers", n);
  HIP_TRY(hipSetDevice(ctx->device));
  mbh_batch *b = new mbh_batch();
  b->ctx = ctx;
  b->hold.set(ctx);
  b->dh = dh;
  auto fail = [&](mbh_status s) {
    batch_free(b);
    return s;
  };
  WalkerC *wc = nullptr;
  double *part = nullptr;
  double2 *dsc = nullptr;
  mbh_status s;
  if ((s = batch_alloc(b, &wc, (size_t)total)) != MBH_OK || (s = batch_alloc(b, &part, (size_t)total * Kmax * 4)) != MBH_OK ||
      (s = batch_alloc(b, &b->redo, 1)) != MBH_OK || (pm_cells && (s = batch_alloc(b, &dsc, pm_cells)) != MBH_OK))
    return fail(s);
  size_t dsc_off = 0;
  std::vector<WorkItem> items(n);
  std::vector<WorkTile> tiles;
  std::vector<WalkerTile> wtiles;
  std::vector<double> cost;
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    WorkItem &it = items[i];
    it = make_item(ctx, refs[i], item_lanes(ctx, refs[i], precs[i]));
    it.prec = precs[i];
    it.theta = theta_dev[i];
    it.wc = wc + off;
    it.lnL = lnL_dev[i];
    it.dhhh = dh_hh_dev ? dh_hh_dev[i] : nullptr;
    it.part = part + off * Kmax * 4;
    it.redo = b->redo;
    it.W = W[i];
    it.offset = off;
    if (refs[i]->pm) {
      it.pm.dsc = dsc + dsc_off;
      dsc_off += (size_t)W[i] * refs[i]->pm_T1 * 3;
    }
    append_tiles(tiles, cost, i, refs[i], it.G, W[i], it.pm.cross_wg);
    append_wtiles(wtiles, i, it);
    off += W[i];
  }
  b->groups = order_tiles(tiles, cost, items.data());
  xcd_align(tiles, b->groups, wtiles, items.data(), n);
  if ((s = batch_alloc(b, &b->items, (size_t)n)) != MBH_OK ||
      (s = batch_alloc(b, &b->tiles, tiles.size())) != MBH_OK ||
      (s = batch_alloc(b, &b->wtiles, wtiles.size())) != MBH_OK)
    return fail(s);
  b->n_wtiles = (int64_t)wtiles.size();
  const unsigned long long zero = 0ull;
  if (hipMemcpy(b->redo, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->items, items.data(), n * sizeof(WorkItem), hipMemcpyHostToDevice) != hipSuccess ||
      (!tiles.empty() && hipMemcpy(b->tiles, tiles.data(), tiles.size() * sizeof(WorkTile), hipMemcpyHostToDevice) != hipSuccess) ||
      (!wtiles.empty() && hipMemcpy(b->wtiles, wtiles.data(), wtiles.size() * sizeof(WalkerTile), hipMemcpyHostToDevice) != hipSuccess))
    return fail(mbh_fail(MBH_EDEVICE, "upload work list"));
  // capture the whole pass once
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(mbh_fail(MBH_EDEVICE, "stream"));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    launch_work(dh, b->n_wtiles, b->groups, b->wtiles, b->items, b->tiles, cs);
    e = hipStreamEndCapture(cs, &b->graph);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) return fail(mbh_fail(MBH_EDEVICE, "graph capture: %s", hipGetErrorString(e)));
  *out = b;
  return MBH_OK;
}

extern "C" mbh_status mbh_batch_create(mbh_ctx *ctx, int n, const mbh_ref *const *refs, const double *const *theta_dev,
                                       const int64_t *W, double *const *lnL_dev, double *const *dh_hh_dev,
                                       mbh_precision prec, mbh_batch **out) {
  if (n < 1) return mbh_fail(MBH_EINVAL, "bad argument");
  std::vector<mbh_precision> precs((size_t)n, prec);
  return mbh_batch_create_prec(ctx, n, refs, theta_dev, W, lnL_dev, dh_hh_dev, precs.data(), out);
}

const WorkItem *batch_device_items(const mbh_batch *b) { return b->items; }

extern "C" mbh_status mbh_batch_launch(mbh_batch *b, hipStream_t st) {
  if (!b) return mbh_fail(MBH_EINVAL, "null batch");
  HIP_TRY(hipSetDevice(b->ctx->device));
  HIP_TRY(hipGraphLaunch(b->exec, st));
  return MBH_OK;
}

extern "C" mbh_status mbh_batch_launch_direct(mbh_batch *b, hipStream_t st) {
  if (!b) return mbh_fail(MBH_EINVAL, "null batch");
  HIP_TRY(hipSetDevice(b->ctx->device));
  launch_work(b->dh, b->n_wtiles, b->groups, b->wtiles, b->items, b->tiles, st);
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

extern "C" mbh_status mbh_batch_launch_stage(mbh_batch *b, int stage, hipStream_t st) {
  if (!b || stage < MBH_STAGE_SETUP || stage > MBH_STAGE_FINISH) return mbh_fail(MBH_EINVAL, "bad batch or stage");
  HIP_TRY(hipSetDevice(b->ctx->device));
  launch_work(b->dh, b->n_wtiles, b->groups, b->wtiles, b->items, b->tiles, st, 1 << (stage - 1));
  HIP_TRY(hipGetLastError());
  return MBH_OK;
}

extern "C" mbh_status mbh_batch_fp64_segments(const mbh_batch *b, uint64_t *count_out) {
  if (!b || !count_out) return mbh_fail(MBH_EINVAL, "null argument");
  HIP_TRY(hipSetDevice(b->ctx->device));
  unsigned long long v = 0;
  HIP_TRY(hipMemcpy(&v, b->redo, sizeof(v), hipMemcpyDeviceToHost));
  *count_out = v;
  return MBH_OK;
}

extern "C" mbh_status mbh_batch_release(mbh_batch *b) {
  if (!b) return MBH_OK;
  (void)hipSetDevice(b->ctx->device);
  (void)hipDeviceSynchronize();
  batch_free(b);
  (void)hipGetLastError();  // teardown errors are not left for the next call to find
  return MBH_OK;
}

// ---------------------------------------------------------------- server
namespace {
using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  int ref = 0;
  int64_t W = 0;  // walkers evaluated (0 for a reference update)
  std::vector<double> theta;
  std::vector<double> lnL, dhhh;
  Clock::time_point t_submit, t_done;
  bool done = false;
  bool failed = false;  // its launch or update could not be issued
  // reference update: the population (theta, lnL_in) it picks from
  const mbh_data *data = nullptr;
  std::vector<double> lnL_in;
  int64_t W_update = 0;
};

// one in-flight batch: device buffers, pinned host staging, stream, event
struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  double *theta_h = nullptr, *res_h = nullptr;  // pinned
  WorkHeader *hdr_h = nullptr;
  WorkItem *items_h = nullptr;
  WorkTile *tiles_h = nullptr;
  WalkerTile *wtiles_h = nullptr;
  // the pinned buffers' device addresses, read and written by k_stage
  const double *theta_hd = nullptr;
  double *res_hd = nullptr;
  const WorkItem *items_hd = nullptr;
  const WorkTile *tiles_hd = nullptr;
  const WalkerTile *wtiles_hd = nullptr;
  double *theta_d = nullptr, *res_d = nullptr;
  WorkItem *items_d = nullptr;
  WorkTile *tiles_d = nullptr;
  WalkerTile *wtiles_d = nullptr;
  int64_t n_wtiles = 0;
  double *part_d = nullptr;        // [cap][Kmax][4]
  WalkerC *wc_d = nullptr;
  std::vector<std::pair<std::shared_ptr<Request>, int64_t>> members;  // request, first walker in the slot
  int64_t walkers = 0;
  std::vector<TileGroup> groups;
  // work-list scratch, kept between batches
  std::vector<WorkTile> tiles;
  std::vector<WalkerTile> wtiles;
  std::vector<double> cost;
  bool busy = false;
};
}  // namespace

struct mbh_server {
  mbh_ctx *ctx = nullptr;
  CtxHold hold;
  std::vector<const mbh_ref *> refs;
  mbh_server_config cfg{};
  int64_t cap_walkers = 0;  // per slot
  int max_items = 0, max_tiles = 0, Kmax = 1;
  size_t bytes_per_walker = 0;
  std::vector<Slot> slots;
  std::vector<std::pair<void *, size_t>> dev_allocs;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
  uint64_t next_id = 1;
  std::atomic<bool> stop{false};
  std::thread thr;
  mbh_server_stats stats{};
  size_t bytes_in_flight = 0;
  int64_t walkers_in_flight = 0;
  std::string thread_error;
  // later batches wait for the last reference update until it has finished
  hipEvent_t barrier = nullptr;
  int updates_in_flight = 0;
};

static void server_free(mbh_server *s) {
  if (s->barrier) (void)hipEventDestroy(s->barrier);
  for (auto &sl : s->slots) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.theta_h) (void)hipHostFree(sl.theta_h);
    if (sl.res_h) (void)hipHostFree(sl.res_h);
    if (sl.hdr_h) (void)hipHostFree(sl.hdr_h);
    if (sl.items_h) (void)hipHostFree(sl.items_h);
    if (sl.tiles_h) (void)hipHostFree(sl.tiles_h);
    if (sl.wtiles_h) (void)hipHostFree(sl.wtiles_h);
  }
  for (auto &a : s->dev_allocs) ctx_free(s->ctx, a.first, a.second);
  delete s;
}

// Take queued requests for a free slot (FIFO, as walker, item and tile
// capacity allow); called with the server lock held.  Only the membership is
// decided here: the work list is built by server_build without the lock.
static bool server_take(mbh_server *s, Slot &sl) {
  sl.members.clear();
  sl.walkers = 0;
  int n_items = 0;
  int64_t n_tiles = 0;
  while (!s->queue.empty()) {
    auto &r = s->queue.front();
    if (r->data) break;  // a reference update: later requests go after it
    const mbh_ref *ref = s->refs[r->ref];
    const int64_t nt = tiles_of(item_lanes(s->ctx, ref, s->cfg.prec), r->W, ref->n_bins + 1);
    if (sl.walkers + r->W > s->cap_walkers || n_items + 1 > s->max_items || n_tiles + nt > s->max_tiles) break;
    n_tiles += nt;
    sl.members.emplace_back(r, sl.walkers);
    sl.walkers += r->W;
    ++n_items;
    s->queue.pop_front();
  }
  return n_items > 0;
}

// Work list of a slot's requests (items, main-pass tiles, walker tiles,
// parameters in the pinned staging buffer); no lock needed: the slot and its
// requests' inputs belong to the server thread until the results are out.
static void server_build(mbh_server *s, Slot &sl) {
  sl.tiles.clear();
  sl.cost.clear();
  sl.wtiles.clear();
  const int n_items = (int)sl.members.size();
  for (int i = 0; i < n_items; ++i) {
    const Request &r = *sl.members[i].first;
    const int64_t off = sl.members[i].second;
    const mbh_ref *ref = s->refs[r.ref];
    const int G = item_lanes(s->ctx, ref, s->cfg.prec);
    WorkItem &it = sl.items_h[i];
    it = make_item(s->ctx, ref, G);
    it.prec = s->cfg.prec;
    it.theta = sl.theta_d + off * 11;
    it.wc = sl.wc_d + off;
    it.part = sl.part_d + off * s->Kmax * 4;
    it.W = r.W;
    it.offset = off;
    // results of item i: lnL at res_d + off (W entries), then dh/hh pairs after the lnL block
    it.lnL = sl.res_d + off;
    it.dhhh = sl.res_d + sl.walkers + 2 * off;
    std::memcpy(sl.theta_h + off * 11, r.theta.data(), r.W * 11 * sizeof(double));
    append_tiles(sl.tiles, sl.cost, i, ref, G, r.W);
  }
  sl.groups = order_tiles(sl.tiles, sl.cost, sl.items_h);
  for (int i = 0; i < n_items; ++i) append_wtiles(sl.wtiles, i, sl.items_h[i]);
  xcd_align(sl.tiles, sl.groups, sl.wtiles, sl.items_h, n_items);
  std::memcpy(sl.tiles_h, sl.tiles.data(), sl.tiles.size() * sizeof(WorkTile));
  std::memcpy(sl.wtiles_h, sl.wtiles.data(), sl.wtiles.size() * sizeof(WalkerTile));
  sl.n_wtiles = (int64_t)sl.wtiles.size();
  *sl.hdr_h = WorkHeader{n_items, (int32_t)sl.tiles.size(), sl.walkers};
}

// Copies of up to four regions of 8-byte words, one grid row per region: a
// batch's inputs from the slot's pinned host buffers into device memory
// (parameters and work tables in one launch), or its results back.  The
// kernel reads and writes the pinned buffers through their device addresses,
// so serving never waits in the runtime's copy path: there a host-to-device
// copy from pinned memory now and then held the scheduler for 6-7 ms.
struct StageCopy {
  const uint64_t *src[4];
  uint64_t *dst[4];
  int64_t words[4];
};
static __global__ __launch_bounds__(256) void k_stage(StageCopy c) {
  const int r = blockIdx.y;
  const uint64_t *__restrict__ src = c.src[r];
  uint64_t *__restrict__ dst = c.dst[r];
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < c.words[r]; i += (int64_t)gridDim.x * 256)
    dst[i] = src[i];
}
static void stage(const StageCopy &c, int n, hipStream_t st) {
  int64_t most = 1;
  for (int r = 0; r < n; ++r) most = std::max(most, c.words[r]);
  const unsigned bx = (unsigned)std::min<int64_t>((most + 255) / 256, 1024);
  hipLaunchKernelGGL(k_stage, dim3(bx, (unsigned)n), dim3(256), 0, st, c);
}
template <typename T>
static const uint64_t *words_of(const T *p) { return (const uint64_t *)p; }
template <typename T>
static uint64_t *words_of(T *p) { return (uint64_t *)p; }
static_assert(sizeof(WorkItem) % 8 == 0 && sizeof(WorkTile) % 8 == 0 && sizeof(WalkerTile) % 8 == 0,
              "staged tables are copied as 8-byte words");

static bool server_launch(mbh_server *s, Slot &sl) {
  const WorkHeader &h = *sl.hdr_h;
  hipStream_t st = sl.st;
  if (s->updates_in_flight > 0 && hipStreamWaitEvent(st, s->barrier, 0) != hipSuccess) return false;
  StageCopy in{};
  in.src[0] = words_of(sl.theta_hd), in.dst[0] = words_of(sl.theta_d), in.words[0] = sl.walkers * 11;
  in.src[1] = words_of(sl.items_hd), in.dst[1] = words_of(sl.items_d);
  in.words[1] = (int64_t)h.n_items * (int64_t)(sizeof(WorkItem) / 8);
  in.src[2] = words_of(sl.tiles_hd), in.dst[2] = words_of(sl.tiles_d);
  in.words[2] = h.n_tiles * (int64_t)(sizeof(WorkTile) / 8);
  in.src[3] = words_of(sl.wtiles_hd), in.dst[3] = words_of(sl.wtiles_d);
  in.words[3] = sl.n_wtiles * (int64_t)(sizeof(WalkerTile) / 8);
  stage(in, 4, st);
  launch_work(true, sl.n_wtiles, sl.groups, sl.wtiles_d, sl.items_d, sl.tiles_d, st);
  StageCopy out{};
  out.src[0] = words_of(sl.res_d), out.dst[0] = words_of(sl.res_hd), out.words[0] = sl.walkers * 3;
  stage(out, 1, st);
  return hipGetLastError() == hipSuccess && hipEventRecord(sl.ev, st) == hipSuccess;
}

// results of a finished batch into its requests' buffers (sized at submit);
// no lock: nobody reads them before server_publish marks the requests done
static void server_copy_results(Slot &sl) {
  const double *lnL = sl.res_h;
  const double *dh = sl.res_h + sl.walkers;
  for (auto &m : sl.members) {
    Request &r = *m.first;
    if (r.data) continue;
    std::memcpy(r.lnL.data(), lnL + m.second, r.W * sizeof(double));
    std::memcpy(r.dhhh.data(), dh + 2 * m.second, r.W * 2 * sizeof(double));
  }
}

// mark a finished slot's requests done (lock held)
static void server_publish(mbh_server *s, Slot &sl) {
  const auto now = Clock::now();
  for (auto &m : sl.members) {
    Request &r = *m.first;
    if (r.data) s->updates_in_flight -= 1;  // the update has finished
    r.t_done = now;
    r.done = true;
  }
  s->stats.completed += sl.members.size();
  s->walkers_in_flight -= sl.walkers;
  s->bytes_in_flight -= (size_t)sl.walkers * s->bytes_per_walker;
  sl.members.clear();
  sl.busy = false;
}

// a slot whose launch or update could not be issued (lock held): its work
// already enqueued has finished (the caller synchronised the slot's stream)
static void server_fail_slot(mbh_server *s, Slot &sl, const char *what) {
  s->thread_error = what;
  const auto now = Clock::now();
  for (auto &m : sl.members) {
    if (m.first->data) s->updates_in_flight -= 1;
    m.first->t_done = now;
    m.first->failed = true;
    m.first->done = true;
  }
  s->walkers_in_flight -= sl.walkers;
  s->bytes_in_flight -= (size_t)sl.walkers * s->bytes_per_walker;
  sl.members.clear();
  sl.busy = false;
  s->cv_done.notify_all();
}

// Issue the reference update held by slot sl: ordered after every batch in
// flight (their events) and before every later batch (the barrier event).
static bool server_issue_update(mbh_server *s, Slot &sl) {
  const std::shared_ptr<Request> &r = sl.members.front().first;
  hipStream_t st = sl.st;
  for (auto &o : s->slots)
    if (&o != &sl && o.busy && hipStreamWaitEvent(st, o.ev, 0) != hipSuccess) return false;
  const int64_t W = r->W_update;
  std::memcpy(sl.theta_h, r->theta.data(), W * 11 * sizeof(double));
  std::memcpy(sl.res_h, r->lnL_in.data(), W * sizeof(double));
  StageCopy in{};
  in.src[0] = words_of(sl.theta_hd), in.dst[0] = words_of(sl.theta_d), in.words[0] = W * 11;
  in.src[1] = words_of(sl.res_hd), in.dst[1] = words_of(sl.res_d), in.words[1] = W;
  stage(in, 2, st);
  if (hipGetLastError() != hipSuccess) return false;
  mbh_ref *ref = const_cast<mbh_ref *>(s->refs[r->ref]);
  if (mbh_ref_refresh(s->ctx, r->data, ref, sl.theta_d, sl.res_d, W, st) != MBH_OK) return false;
  return hipEventRecord(s->barrier, st) == hipSuccess && hipEventRecord(sl.ev, st) == hipSuccess;
}

// The scheduler thread.  Slot state, staging buffers and the in-flight
// update count belong to this thread; the queue, request flags and
// statistics are shared under s->mu, which is held only to retire finished
// batches, to take queued work and to record failures.  Building the work
// lists, copying parameters and results and issuing launches run without
// it, so submitting and waiting threads are not held up by them.
static void server_loop(mbh_server *s) {
  (void)hipSetDevice(s->ctx->device);
  using Sec = std::chrono::duration<double>;
  std::vector<Slot *> finished, filled;
  while (!s->stop.load()) {
    // 1. finished batches: results out without the lock
    finished.clear();
    for (auto &sl : s->slots)
      if (sl.busy && hipEventQuery(sl.ev) == hipSuccess) finished.push_back(&sl);
    const auto t0 = Clock::now();
    for (Slot *sl : finished) server_copy_results(*sl);
    const auto t1 = Clock::now();
    // 2. retire them and take queued work for the free slots
    filled.clear();
    bool any_busy = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->stats.host_complete_s += Sec(t1 - t0).count();
      for (Slot *sl : finished) server_publish(s, *sl);
      if (!finished.empty()) s->cv_done.notify_all();
      for (auto &sl : s->slots) {
        if (sl.busy || s->queue.empty()) continue;
        if (s->queue.front()->data) {
          sl.members.clear();
          sl.members.emplace_back(s->queue.front(), 0);
          s->queue.pop_front();
          sl.walkers = 0;
        } else if (!server_take(s, sl)) {
          continue;
        } else {
          s->walkers_in_flight += sl.walkers;
          s->bytes_in_flight += (size_t)sl.walkers * s->bytes_per_walker;
          s->stats.max_walkers_in_flight = std::max<uint64_t>(s->stats.max_walkers_in_flight, s->walkers_in_flight);
          s->stats.max_bytes_in_flight = std::max<uint64_t>(s->stats.max_bytes_in_flight, s->bytes_in_flight);
          s->stats.walkers += sl.walkers;
        }
        s->stats.batches += 1;
        sl.busy = true;
        filled.push_back(&sl);
      }
      for (auto &sl : s->slots) any_busy |= sl.busy;
      if (!s->queue.empty() && filled.empty()) s->stats.admission_waits += 1;
      if (finished.empty() && filled.empty() && !any_busy) {
        s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
        continue;
      }
    }
    // 3. build and issue the filled slots without the lock
    for (Slot *sl : filled) {
      const bool update = sl->members.front().first->data != nullptr;
      const auto b0 = Clock::now();
      bool ok;
      if (update) {
        s->updates_in_flight += 1;
        ok = server_issue_update(s, *sl);
      } else {
        server_build(s, *sl);
        ok = server_launch(s, *sl);
      }
      const auto b1 = Clock::now();
      if (!ok) (void)hipStreamSynchronize(sl->st);  // work already enqueued finishes before the slot is reused
      std::lock_guard<std::mutex> g(s->mu);
      s->stats.host_build_s += Sec(b1 - b0).count();
      if (!ok) server_fail_slot(s, *sl, update ? "reference update failed" : "launch failed");
    }
    // 4. nothing changed: let the submitting and waiting threads run
    if (finished.empty() && filled.empty()) std::this_thread::yield();
  }
}

extern "C" mbh_status mbh_server_create(mbh_ctx *ctx, int n_refs, const mbh_ref *const *refs,
                                        const mbh_server_config *cfg, mbh_server **out) {
  if (!ctx || !refs || !cfg || !out || n_refs < 1) return mbh_fail(MBH_EINVAL, "bad argument");
  *out = nullptr;
  if (cfg->max_inflight < 1 || cfg->max_inflight > 8 || cfg->max_batch_walkers < 1)
    return mbh_fail(MBH_EINVAL, "max_inflight in [1, 8] and max_batch_walkers >= 1 required");
  if (cfg->prec != MBH_FP64 && cfg->prec != MBH_MIXED) return mbh_fail(MBH_EINVAL, "bad precision");
  for (int i = 0; i < n_refs; ++i) {
    if (!refs[i] || refs[i]->ctx != ctx) return mbh_fail(MBH_EINVAL, "reference %d invalid", i);
    if (refs[i]->pm) return mbh_fail(MBH_EINVAL, "reference %d: per-mode references are not served", i);
  }
  HIP_TRY(hipSetDevice(ctx->device));
  mbh_server *s = new mbh_server();
  s->ctx = ctx;
  s->hold.set(ctx);
  s->refs.assign(refs, refs + n_refs);
  s->cfg = *cfg;
  for (int i = 0; i < n_refs; ++i) {
    s->Kmax = std::max(s->Kmax, flat_slots(refs[i]->n_bins + 1));
  }
  // inputs, outputs, walker constants and the per-walker partial sums
  s->bytes_per_walker = 11 * sizeof(double) + 3 * sizeof(double) + sizeof(WalkerC) + 4 * sizeof(double) * s->Kmax;
  int64_t cap = cfg->max_batch_walkers;
  if (cfg->hbm_budget_bytes) {
    int64_t by_budget = (int64_t)(cfg->hbm_budget_bytes / (cfg->max_inflight * s->bytes_per_walker));
    cap = std::min(cap, by_budget);
  }
  if (cap < 1) {
    delete s;
    return mbh_fail(MBH_ENOMEM, "HBM budget too small for one walker per slot");
  }
  s->cap_walkers = cap;
  s->max_items = (int)std::min<int64_t>(cap, 4096);
  {
    // tiles of a full slot: flattened chunks (E / (63 kWaves) per walker) or
    // lane groups (at most one walker per lane), plus one partial tile per item
    int Emax = 2;
    for (int i = 0; i < n_refs; ++i) Emax = std::max(Emax, refs[i]->n_bins + 1);
    const int64_t per_walker_x = std::max<int64_t>(kBlock, (Emax + kChunk * kWaves - 1) / (kChunk * kWaves) * kBlock);
    s->max_tiles = (int)std::min<int64_t>(cap * per_walker_x / kBlock + 2 * s->max_items, INT32_MAX / 2);
  }
  s->slots.resize(cfg->max_inflight);
  auto dalloc = [&](void **p, size_t bytes) {
    mbh_status st = ctx_alloc(ctx, p, bytes);
    if (st == MBH_OK) s->dev_allocs.emplace_back(*p, bytes);
    return st;
  };
  for (auto &sl : s->slots) {
    mbh_status st;
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&sl.theta_h, cap * 11 * sizeof(double), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&sl.res_h, cap * 3 * sizeof(double), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&sl.hdr_h, sizeof(WorkHeader), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&sl.items_h, s->max_items * sizeof(WorkItem), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&sl.tiles_h, s->max_tiles * sizeof(WorkTile), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc((void **)&sl.wtiles_h, (cap / kWalkerTile + s->max_items + 1) * sizeof(WalkerTile),
                      hipHostMallocCoherent) != hipSuccess ||
        hipHostGetDevicePointer((void **)&sl.theta_hd, sl.theta_h, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&sl.res_hd, sl.res_h, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&sl.items_hd, sl.items_h, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&sl.tiles_hd, sl.tiles_h, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&sl.wtiles_hd, sl.wtiles_h, 0) != hipSuccess) {
      server_free(s);
      return mbh_fail(MBH_EDEVICE, "server host resources");
    }
    if ((st = dalloc((void **)&sl.theta_d, cap * 11 * sizeof(double))) != MBH_OK ||
        (st = dalloc((void **)&sl.res_d, cap * 3 * sizeof(double))) != MBH_OK ||
        (st = dalloc((void **)&sl.wtiles_d, (cap / kWalkerTile + s->max_items + 1) * sizeof(WalkerTile))) != MBH_OK ||
        (st = dalloc((void **)&sl.items_d, s->max_items * sizeof(WorkItem))) != MBH_OK ||
        (st = dalloc((void **)&sl.tiles_d, s->max_tiles * sizeof(WorkTile))) != MBH_OK ||
        (st = dalloc((void **)&sl.part_d, cap * s->Kmax * 4 * sizeof(double))) != MBH_OK ||
        (st = dalloc((void **)&sl.wc_d, cap * sizeof(WalkerC))) != MBH_OK) {
      server_free(s);
      return st;
    }
  }
  if (hipEventCreateWithFlags(&s->barrier, hipEventDisableTiming) != hipSuccess) {
    server_free(s);
    return mbh_fail(MBH_EDEVICE, "server event");
  }
  s->thr = std::thread(server_loop, s);
  *out = s;
  return MBH_OK;
}

extern "C" mbh_status mbh_server_submit(mbh_server *s, int ref_index, const double *theta_host, int64_t W,
                                        uint64_t *request_id) {
  if (!s || !theta_host || !request_id || W < 1) return mbh_fail(MBH_EINVAL, "bad argument");
  if (ref_index < 0 || ref_index >= (int)s->refs.size()) return mbh_fail(MBH_EINVAL, "reference index %d", ref_index);
  if (W > s->cap_walkers)
    return mbh_fail(MBH_EAGAIN, "request of %lld walkers exceeds the per-batch capacity %lld", (long long)W,
                    (long long)s->cap_walkers);
  auto r = std::make_shared<Request>();
  r->ref = ref_index;
  r->W = W;
  r->theta.assign(theta_host, theta_host + W * 11);
  r->lnL.resize(W);
  r->dhhh.resize(2 * W);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(s->mu);
    r->id = s->next_id++;
    s->live[r->id] = r;
    s->queue.push_back(r);
    s->stats.submitted += 1;
  }
  s->cv_work.notify_one();
  *request_id = r->id;
  return MBH_OK;
}

extern "C" mbh_status mbh_server_refresh(mbh_server *s, int ref_index, const mbh_data *data,
                                         const double *theta_host, const double *lnL_host, int64_t W,
                                         uint64_t *request_id) {
  if (!s || !data || !theta_host || !lnL_host || !request_id || W < 1) return mbh_fail(MBH_EINVAL, "bad argument");
  if (ref_index < 0 || ref_index >= (int)s->refs.size()) return mbh_fail(MBH_EINVAL, "reference index %d", ref_index);
  const mbh_ref *ref = s->refs[ref_index];
  if (data->ctx != s->ctx || data->n_chan != ref->n_chan || data->n_f != ref->n_f || data->f0 != ref->f0 ||
      data->df != ref->df || data->t_obs != ref->t_obs)
    return mbh_fail(MBH_EINVAL, "data grid differs from the one the reference was built on");
  if (W > s->cap_walkers)
    return mbh_fail(MBH_EAGAIN, "update population of %lld walkers exceeds the per-batch capacity %lld",
                    (long long)W, (long long)s->cap_walkers);
  auto r = std::make_shared<Request>();
  r->ref = ref_index;
  r->W = 0;
  r->data = data;
  r->W_update = W;
  r->theta.assign(theta_host, theta_host + W * 11);
  r->lnL_in.assign(lnL_host, lnL_host + W);
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> g(s->mu);
    r->id = s->next_id++;
    s->live[r->id] = r;
    s->queue.push_back(r);
    s->stats.submitted += 1;
  }
  s->cv_work.notify_one();
  *request_id = r->id;
  return MBH_OK;
}

extern "C" mbh_status mbh_server_wait(mbh_server *s, uint64_t id, int timeout_ms, double *lnL_host,
                                      double *dh_hh_host, int64_t capacity, double *latency_s_out) {
  if (!s) return mbh_fail(MBH_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->live.find(id);
  if (it == s->live.end()) return mbh_fail(MBH_ENOTFOUND, "request %llu", (unsigned long long)id);
  std::shared_ptr<Request> r = it->second;
  if ((lnL_host || dh_hh_host) && capacity < r->W)
    return mbh_fail(MBH_EINVAL, "request %llu holds %lld walkers, the output buffers %lld", (unsigned long long)id,
                    (long long)r->W, (long long)capacity);
  auto ready = [&] { return r->done; };
  if (timeout_ms < 0) s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return MBH_EAGAIN;
  if (r->failed) {
    s->live.erase(it);
    return mbh_fail(MBH_EDEVICE, "server: %s", s->thread_error.c_str());
  }
  if (lnL_host) std::memcpy(lnL_host, r->lnL.data(), r->W * sizeof(double));
  if (dh_hh_host) std::memcpy(dh_hh_host, r->dhhh.data(), r->W * 2 * sizeof(double));
  if (latency_s_out) *latency_s_out = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  s->live.erase(it);
  return MBH_OK;
}

// Submit and collect a request trace from native threads: the calling thread
// submits request i when the steady clock reaches its arrival time, a second
// thread takes the results in request order as they finish.
extern "C" mbh_status mbh_server_replay(mbh_server *s, const mbh_request_spec *reqs, int64_t n,
                                        const double *theta_host, int64_t theta_rows, double *latency_s,
                                        double *submit_lag_s, double *lnL_host, double *wall_s) {
  if (!s || !reqs || n < 1 || !theta_host || !latency_s) return mbh_fail(MBH_EINVAL, "bad argument");
  std::vector<int64_t> out_off((size_t)n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const mbh_request_spec &q = reqs[i];
    if (!(q.t_arrival_s >= 0.0) || (i > 0 && q.t_arrival_s < reqs[i - 1].t_arrival_s))
      return mbh_fail(MBH_EINVAL, "request %lld: arrival times must be finite, >= 0 and non-decreasing", (long long)i);
    if (q.ref_index < 0 || q.ref_index >= (int)s->refs.size() || q.W < 1 || q.W > s->cap_walkers ||
        q.theta_row < 0 || q.theta_row + q.W > theta_rows)
      return mbh_fail(MBH_EINVAL, "request %lld: bad reference, walker count or theta rows", (long long)i);
    out_off[i + 1] = out_off[i] + q.W;
  }
  using Sec = std::chrono::duration<double>;
  std::vector<uint64_t> ids((size_t)n, 0);
  std::vector<std::atomic<int>> posted((size_t)n);
  for (auto &p : posted) p.store(0);
  std::atomic<int64_t> submitted{0};
  mbh_status failure = MBH_OK;
  std::string failure_msg;
  const auto t0 = Clock::now();
  std::thread collector([&] {
    for (int64_t i = 0; i < n; ++i) {
      while (!posted[i].load(std::memory_order_acquire)) {
        if (posted[i].load() < 0) return;
        std::this_thread::yield();
      }
      if (posted[i].load() < 0) return;
      std::shared_ptr<Request> r;
      {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->live.find(ids[i]);
        if (it == s->live.end()) continue;
        r = it->second;
        s->cv_done.wait(lk, [&] { return r->done; });
        s->live.erase(it);
      }
      const auto arrival = t0 + std::chrono::duration_cast<Clock::duration>(Sec(reqs[i].t_arrival_s));
      latency_s[i] = r->failed ? NAN : Sec(r->t_done - arrival).count();
      if (submit_lag_s) submit_lag_s[i] = Sec(r->t_submit - arrival).count();
      if (lnL_host) {
        if (r->failed) std::fill(lnL_host + out_off[i], lnL_host + out_off[i + 1], NAN);
        else std::copy(r->lnL.begin(), r->lnL.end(), lnL_host + out_off[i]);
      }
    }
  });
  int64_t i = 0;
  for (; i < n; ++i) {
    const auto arrival = t0 + std::chrono::duration_cast<Clock::duration>(Sec(reqs[i].t_arrival_s));
    for (;;) {
      const auto now = Clock::now();
      if (now >= arrival) break;
      if (arrival - now > std::chrono::microseconds(300)) std::this_thread::sleep_for(std::chrono::microseconds(100));
      else std::this_thread::yield();
    }
    mbh_status st = mbh_server_submit(s, reqs[i].ref_index, theta_host + reqs[i].theta_row * 11, reqs[i].W, &ids[i]);
    if (st != MBH_OK) {
      failure = st;
      failure_msg = mbh_last_error();
      break;
    }
    posted[i].store(1, std::memory_order_release);
  }
  for (int64_t k = i; k < n; ++k) posted[k].store(-1);
  collector.join();
  if (wall_s) *wall_s = Sec(Clock::now() - t0).count();
  if (failure != MBH_OK) return mbh_fail(failure, "request %lld: %s", (long long)i, failure_msg.c_str());
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (!s->thread_error.empty()) return mbh_fail(MBH_EDEVICE, "server: %s", s->thread_error.c_str());
  }
  return MBH_OK;
}

extern "C" mbh_status mbh_server_get_stats(const mbh_server *s, mbh_server_stats *out) {
  if (!s || !out) return mbh_fail(MBH_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(const_cast<mbh_server *>(s)->mu);
  *out = s->stats;
  return MBH_OK;
}

extern "C" mbh_status mbh_server_destroy(mbh_server *s) {
  if (!s) return MBH_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop.store(true);
  }
  s->cv_work.notify_all();
  if (s->thr.joinable()) s->thr.join();
  (void)hipSetDevice(s->ctx->device);
  server_free(s);
  (void)hipGetLastError();  // teardown errors are not left for the next call to find
  return MBH_OK;
}
