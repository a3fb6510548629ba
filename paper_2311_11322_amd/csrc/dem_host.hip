// dem_host.hip -- host runtime behind the C-ABI of include/dem.h.
//
// Owns each system's device buffers (through the caller's allocator), the
// device table of piles, the static work lists, and one captured HIP graph
// per batch that replays a whole step.  No host synchronisation happens
// inside a step; dem_step reads back one small status record per call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "dem.h"
#include "dem_internal.h"

using namespace dem;

namespace {

thread_local std::string g_error = "no error";

constexpr int kDefaultContacts = 8;
constexpr int kFindContactsCap = 64;

std::string hip_msg(hipError_t e, const char* what) {
  return std::string(what) + ": " + hipGetErrorString(e);
}

struct Allocator {
  dem_allocator user{};
  bool has_user = false;
  void* alloc(size_t n) const {
    if (n == 0) n = 256;
    n = (n + 255) & ~size_t(255);
    if (has_user) return user.alloc(n, user.ctx);
    void* p = nullptr;
    if (hipMalloc(&p, n) != hipSuccess) return nullptr;
    return p;
  }
  void release(void* p) const {
    if (!p) return;
    if (has_user) user.free(p, user.ctx);
    else (void)hipFree(p);
  }
};

size_t round256(size_t n) { return (n + 255) & ~size_t(255); }

int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

// Device footprint of one system, byte for byte what alloc_pile allocates.
struct Sizes {
  int64_t na, ns, cap, cells, g_tile, g_nt, g_np, n_rblk;
  int g_form;                // 1 super-tile pairs, 2 per-target
  bool grav;
  bool tree;
  int64_t tree_nodes;        // all levels of the pyramid
  int precision;
};

// Cells per axis of a periodic cube of side L: as many as fit with a side of
// at least cell_min (with a relative margin against rounding), at least one,
// and no more than the Morton table holds.
int periodic_cells(double L, double cell_min, int bits) {
  const double ratio = L / (cell_min * (1.0 + 1e-12));
  int n = ratio >= 1.0 ? (int)std::min(std::floor(ratio), 1e9) : 1;
  return std::max(1, std::min(n, 1 << bits));
}

// Spheres much larger than the rest -- above twice the median radius, if
// there are at most kMaxBig of them -- are searched separately, so that the
// cells can be sized for the others (a boulder among grains).
void split_big(const double* radius, int64_t ns, double* s_cut, double* s_small, int* n_big) {
  std::vector<double> r(radius, radius + ns);
  std::nth_element(r.begin(), r.begin() + ns / 2, r.end());
  const double cut = 2.0 * r[ns / 2];
  int64_t nb = 0;
  double small = 0.0, all = 0.0;
  for (int64_t i = 0; i < ns; ++i) {
    all = std::max(all, radius[i]);
    if (radius[i] > cut) ++nb;
    else small = std::max(small, radius[i]);
  }
  if (nb == 0 || nb > kMaxBig) {
    *s_cut = INFINITY;
    *s_small = all;
    *n_big = 0;
  } else {
    *s_cut = cut;
    *s_small = small;
    *n_big = (int)nb;
  }
}

int choose_bits(int64_t ns) {
  // at least two cells per sphere, 2..10 bits per axis
  int b = (ceil_log2(uint64_t(2 * ns)) + 2) / 3;
  return std::min(10, std::max(2, b));
}

int default_tile(int precision) {
  int t[8];
  gravity_tiles(precision, t);
  return t[0];
}

bool tile_supported(int precision, int tile) {
  int t[8];
  const int n = gravity_tiles(precision, t);
  for (int k = 0; k < n; ++k)
    if (t[k] == tile) return true;
  return false;
}

Sizes pile_sizes(const dem_params& p, int64_t na, int64_t ns, int c_max, int tile,
                 int form = 0) {
  Sizes z;
  z.na = na;
  z.ns = ns;
  z.cap = int64_t(c_max) * ns;
  z.cells = int64_t(1) << (3 * choose_bits(ns));
  z.grav = p.G != 0.0;
  z.tree = z.grav && p.gravity_tree;
  z.tree_nodes = z.tree ? ((z.cells << 3) - 1) / 7 : 0;
  z.precision = p.precision;
  z.g_tile = tile > 0 ? tile : default_tile(p.precision);
  z.g_nt = (ns + z.g_tile - 1) / z.g_tile;
  // the exact sum's form: super-tile pairs (one partial per super-tile)
  // unless asked otherwise or their partials would exceed kSymPartialMax
  const int64_t pair_span = (z.g_nt + kGravSlots - 1) / kGravSlots;
  const int64_t pair_np = (z.g_nt + pair_span - 1) / pair_span;
  const int64_t part_bytes = pair_np * 3 * ns * (p.precision == 1 ? 4 : 8);
  z.g_form = form != 0 ? form : (part_bytes > kSymPartialMax ? 2 : 1);
  if (z.g_form == 2) {
    const int64_t span = (z.g_nt + kGravSplits - 1) / kGravSplits;
    z.g_np = (z.g_nt + span - 1) / span;
  } else {
    z.g_np = pair_np;
  }
  z.n_rblk = (ns + kBlock - 1) / kBlock;
  return z;
}

struct BufList {
  std::vector<std::pair<void**, size_t>> req;
  template <typename T>
  void add(T** p, int64_t count) {
    req.push_back({reinterpret_cast<void**>(p), round256(size_t(std::max<int64_t>(count, 1)) * sizeof(T))});
  }
  size_t total() const {
    size_t t = 0;
    for (auto& r : req) t += r.second;
    return t;
  }
};

void plan_pile(PileDev& h, const Sizes& z, BufList& L) {
  const int64_t na = z.na, ns = z.ns, cap = z.cap;
  L.add(&h.first, na);
  L.add(&h.count, na);
  L.add(&h.M, na);
  L.add(&h.I, 3 * na);
  for (int k = 0; k < 2; ++k) {
    L.add(&h.rA[k], 3 * na);
    L.add(&h.vA[k], 3 * na);
    L.add(&h.aA[k], 3 * na);
    L.add(&h.NA[k], 3 * na);
    L.add(&h.q[k], 4 * na);
    L.add(&h.wb[k], 3 * na);
  }
  L.add(&h.wA, 3 * na);
  L.add(&h.vpred, 3 * na);
  L.add(&h.b, 3 * ns);
  L.add(&h.s, ns);
  L.add(&h.m, ns);
  L.add(&h.agg, ns);
  L.add(&h.r, 3 * ns);
  L.add(&h.v, 3 * ns);
  L.add(&h.F, 3 * ns);
  L.add(&h.tau, 3 * ns);
  L.add(&h.key, ns);
  L.add(&h.sidx, ns);
  L.add(&h.sidx_raw, ns);
  L.add(&h.slot, ns);
  L.add(&h.xs, 4 * ns);
  L.add(&h.xg, ns);
  L.add(&h.sid, ns);
  if (z.grav) {
    L.add(reinterpret_cast<double**>(&h.jrec), 8 * ns);
    L.add(&h.gacc, 3 * ns);
    if (z.tree) {
      L.add(&h.tmom, kMom * z.tree_nodes);
      L.add(&h.traw, kRaw * z.tree_nodes);
      L.add(&h.tpart, 64 * 3 * ns);
      L.add(&h.tbox, 6 * ((ns + 63) / 64));
    } else {
      // partials: g_np x 3 x ns values (FP64, or FP32 in the FP32-force form)
      const int64_t part_vals = z.g_np * 3 * ns;
      L.add(&h.ganchor, 4 * z.g_nt);
      L.add(reinterpret_cast<double**>(&h.gpart), z.precision == 1 ? (part_vals + 1) / 2 : part_vals);
    }
  }
  L.add(&h.bpart, kBbox * z.n_rblk);
  L.add(&h.ppart, 3 * z.n_rblk);
  L.add(&h.grid, 1);
  L.add(&h.cell_cnt, z.cells + 1);          // + the cell of the big spheres
  L.add(&h.cell_start, z.cells + 2);
  L.add(&h.run_cache, 2 * kRunCache * ns);
  L.add(&h.cnt_up, ns);
  L.add(&h.cnt_lo, ns);
  L.add(&h.up_off[0], ns + 1);
  L.add(&h.up_off[1], ns + 1);
  L.add(&h.lo_off, ns + 1);
  L.add(&h.pair_j[0], cap);
  L.add(&h.pair_j[1], cap);
  L.add(&h.hist[0], kHist * cap);
  L.add(&h.hist[1], kHist * cap);
  L.add(&h.lo_nbr, cap);
}

double dashpot_factor(double eps) {
  const double le = std::log(eps);
  return -2.0 * le / std::sqrt(M_PI * M_PI + le * le);
}

}  // namespace

// ---------------------------------------------------------------------------
// batches: the device table of piles, work lists and the step graph
// ---------------------------------------------------------------------------

struct Batch {
  std::vector<dem_sim*> members;
  PileDev* d_table = nullptr;
  int table_cap = 0;
  std::vector<void*> meta;          // hipMalloc'ed work lists (freed on rebuild)
  WorkItem* wl_agg = nullptr;
  int n_agg_blk = 0;
  WorkItem* wl_sph = nullptr;
  WorkItem* wl_big = nullptr;                // (pile, k-th big sphere)
  int n_big_blk = 0;
  WorkItem* wl_tree[11] = {};                // per pyramid level: (pile, first node)
  int n_tree[11] = {};
  bool any_tree = false;
  bool tree_order[2] = {false, false};       // some tree pile of order 2, 4
  unsigned tree_leaf_levels = 0;             // bit l: level l is some tree pile's finest
  int n_sph_blk = 0;
  // gravity super-tile pairs, grouped by tile size (one launch per group)
  GravItem* gl[3] = {nullptr, nullptr, nullptr};
  int n_grav[3] = {0, 0, 0};
  // super-tile pairs of piles with more than kGravSlots tiles, same grouping
  GravItem* gm[3] = {nullptr, nullptr, nullptr};
  int n_gmulti[3] = {0, 0, 0};
  // per-target form: (target tile, source split) items, same grouping
  GravItem* gs[3] = {nullptr, nullptr, nullptr};
  int n_gsplit[3] = {0, 0, 0};
  int grav_tile[3] = {0, 0, 0};
  int n_grav_groups = 0;
  bool any_grav = false;
  bool any_direct = false;                   // some pile with the exact sum
  bool reduce_stage = false;                 // member reduction through LDS
  // piles whose whole step runs in one workgroup (k_fused): with gravity
  // (parts 1 and 2 around the gravity kernels) and without (part 3)
  int32_t* pl_fused_g = nullptr;
  int n_fused_g = 0;
  int32_t* pl_fused_ng = nullptr;
  int n_fused_ng = 0;
  int n_staged = 0;                          // piles stepped by the staged kernels
  WorkItem* wl_grav = nullptr;               // spheres of every pile with gravity
  int n_grav_blk = 0;
  WorkItem* wl_agg_all = nullptr;            // aggregates of every pile (set-up)
  int n_agg_all_blk = 0;
  bool all_soft = true;
  ScanSeg* seg_cells = nullptr;
  ScanItem* item_cells = nullptr;
  uint32_t* sums_cells = nullptr;
  int n_seg_cells = 0, n_item_cells = 0, max_items_cells = 0;
  ScanSeg* seg_pairs = nullptr;
  ScanItem* item_pairs = nullptr;
  uint32_t* sums_pairs = nullptr;
  int n_seg_pairs = 0, n_item_pairs = 0, max_items_pairs = 0;
  hipGraphExec_t graph = nullptr;
  hipGraph_t graph_def = nullptr;
  // gravity runs on a second stream beside the contact search and forces
  // (fork after the cell sort, join before the member reduction)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool dirty = true;
  ContactParams cp{};
  int precision = 0;
};

struct dem_sim {
  dem_params prm{};
  Allocator alloc;
  hipStream_t stream = nullptr;
  std::string err = "no error";
  // device storage
  PileDev h{};                       // host mirror of this system's table entry
  std::vector<void*> bufs;
  size_t bytes = 0;
  Sizes sz{};
  int c_max = kDefaultContacts;
  bool has_aggs = false;
  bool stepped = false;
  dem_forcing forcing{};
  // where the authoritative copy of the table entry lives
  Batch own;                         // standalone batch of one
  dem_engine* engine = nullptr;
  int engine_slot = -1;
  dem_status last_status = DEM_OK;
  dem_tuning tune{0, 1.0, 0, 0, 0};
  // per-kernel timing: 0 off, 1 launches one after another with events
  // between kernels, 2 launches ordered as in the graph with events around
  // the gravity stage only
  int profiling = 0;
  std::vector<hipEvent_t> events;
  std::vector<double> prof_ms;
  int64_t prof_steps = 0;
};

struct dem_engine {
  size_t budget = 0, used = 0;
  hipStream_t stream = nullptr;
  Batch batch;
  std::string err = "no error";
  // per-kernel timing, as for a standalone system
  bool profiling = false;
  std::vector<hipEvent_t> events;
  std::vector<double> prof_ms;
  int64_t prof_steps = 0;
};

namespace {

dem_status fail(dem_sim* s, dem_status code, const std::string& msg) {
  g_error = msg;
  if (s) s->err = msg;
  return code;
}

// The library's HIP runtime must see a device before anything is allocated:
// a process that also holds PyTorch (which carries its own HIP runtime) has to
// initialise PyTorch first, or this runtime may come up without a GPU.
dem_status require_device(dem_sim* s) {
  int n = 0;
  const hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0)
    return fail(s, DEM_ERR_DEVICE,
                std::string("no HIP device visible to the library's runtime (") +
                    (e != hipSuccess ? hipGetErrorString(e) : "0 devices") +
                    "); in a process that uses PyTorch, initialise PyTorch's GPU before "
                    "loading this library");
  return DEM_OK;
}

#define HIPCHK(sim, call)                                                   \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) return fail((sim), DEM_ERR_DEVICE, hip_msg(e_, #call)); \
  } while (0)

void free_meta(Batch& b) {
  for (void* p : b.meta) (void)hipFree(p);
  b.meta.clear();
  if (b.graph) (void)hipGraphExecDestroy(b.graph);
  if (b.graph_def) (void)hipGraphDestroy(b.graph_def);
  b.graph = nullptr;
  b.graph_def = nullptr;
}

template <typename T>
hipError_t upload(Batch& b, T** dst, const std::vector<T>& src, hipStream_t st) {
  *dst = nullptr;
  if (src.empty()) return hipSuccess;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  b.meta.push_back(p);
  *dst = static_cast<T*>(p);
  return hipMemcpyAsync(p, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

// Rebuild work lists and scan segments of a batch from its members; the
// device table entries must already be in place at slots 0..n-1.
dem_status rebuild(Batch& b, hipStream_t st, dem_sim* errsim) {
  free_meta(b);
  std::vector<WorkItem> wa, wsph, wbig, wtree[11], wgrav, wall;
  std::vector<int32_t> pfg, pfng;
  std::vector<GravItem> glg[3], gmg[3], gsg[3];
  std::vector<std::pair<int64_t, GravItem>> gmw[3];
  int tiles[3] = {0, 0, 0};
  int n_groups = 0;
  std::vector<ScanSeg> sc, sp;
  std::vector<ScanItem> ic, ip;
  b.any_grav = false;
  b.any_direct = false;
  b.any_tree = false;
  b.tree_order[0] = b.tree_order[1] = false;
  b.tree_leaf_levels = 0;
  b.all_soft = true;
  int64_t tot_na = 0;
  b.n_staged = 0;
  for (int p = 0; p < (int)b.members.size(); ++p) {
    const dem_sim* s = b.members[p];
    const PileDev& h = s->h;
    if (h.G != 0.0)
      for (int i = 0; i < h.ns; i += kBlock) wgrav.push_back({p, i});
    for (int a = 0; a < h.na; a += kBlock) wall.push_back({p, a});
    if (h.fused) {
      (h.G != 0.0 ? pfg : pfng).push_back(p);
    } else {
      b.n_staged++;
      for (int a = 0; a < h.na; a += kBlock) wa.push_back({p, a});
      tot_na += h.na;
      for (int i = 0; i < h.ns; i += kBlock) wsph.push_back({p, i});
      for (int k = 0; k < h.n_big; ++k) wbig.push_back({p, k});
    }
    if (h.G != 0.0 && h.tree) {
      b.any_grav = true;
      b.any_tree = true;
      b.tree_order[h.tree_order == 4 ? 1 : 0] = true;
      b.tree_leaf_levels |= 1u << h.bits;
      for (int l = 0; l <= h.bits; ++l)
        // the finest level: 256 nodes per block; above it eight lanes per node
        for (int64_t q = 0, step = l == h.bits ? kBlock : kBlock / 8; q < (int64_t(1) << (3 * l));
             q += step)
          wtree[l].push_back({p, (int32_t)q});
    } else if (h.G != 0.0) {
      b.any_grav = true;
      b.any_direct = true;
      if (!(h.soft_frac > 0.0)) b.all_soft = false;
      // every super-tile pair (si <= sj) of the pile: each unordered pair
      // once; or every (target tile, source split) of the per-target form
      int g = 0;
      while (g < n_groups && tiles[g] != h.g_tile) ++g;
      if (g == n_groups) tiles[n_groups++] = h.g_tile;
      if (h.g_form == 2) {
        const int grp = 64 * gravity_split_ipt(b.precision, h.g_tile);
        const int n_grp = (h.ns + grp - 1) / grp;
        for (int tg = 0; tg < n_grp; ++tg)
          for (int sp = 0; sp < h.g_np; ++sp) gsg[g].push_back({p, tg, sp, 0});
      } else {
        if (h.g_np == h.g_nt) {
          for (int si = 0; si < h.g_np; ++si)
            for (int sj = si; sj < h.g_np; ++sj) glg[g].push_back({p, si, sj, 0});
        } else {
          // super-tiles of several tiles: items weighted by their tile pairs
          const int span = (h.g_nt + kGravSlots - 1) / kGravSlots;
          auto tiles = [&](int sp) { return (int64_t)std::min(span, h.g_nt - sp * span); };
          for (int si = 0; si < h.g_np; ++si)
            for (int sj = si; sj < h.g_np; ++sj)
              gmw[g].push_back({si == sj ? tiles(si) * (tiles(si) + 1) / 2 : tiles(si) * tiles(sj),
                                GravItem{p, si, sj, 0}});
        }
      }
    }
    // cell-count scan of this pile
    auto add_seg = [](std::vector<ScanSeg>& segs, std::vector<ScanItem>& items, const uint32_t* in,
                      uint32_t* out0, uint32_t* out1, const int32_t* par, int64_t n) {
      ScanSeg g{};
      g.in = in;
      g.out_pp[0] = out0;
      g.out_pp[1] = out1;
      g.parity = par;
      g.n = (int32_t)n;
      g.item0 = (int32_t)items.size();
      g.n_items = (int32_t)((n + kScanChunk - 1) / kScanChunk);
      for (int c = 0; c < g.n_items; ++c) items.push_back({(int32_t)segs.size(), c});
      segs.push_back(g);
    };
    if (h.fused) continue;
    PileDev* dentry = b.d_table + p;
    add_seg(sc, ic, h.cell_cnt, h.cell_start, h.cell_start, nullptr, s->sz.cells + 1);
    add_seg(sp, ip, h.cnt_up, h.up_off[0], h.up_off[1], &dentry->parity, h.ns);
    add_seg(sp, ip, h.cnt_lo, h.lo_off, h.lo_off, nullptr, h.ns);
  }
  HIPCHK(errsim, upload(b, &b.wl_agg, wa, st));
  HIPCHK(errsim, upload(b, &b.wl_grav, wgrav, st));
  HIPCHK(errsim, upload(b, &b.wl_agg_all, wall, st));
  b.n_agg_all_blk = (int)wall.size();
  b.n_grav_blk = (int)wgrav.size();
  HIPCHK(errsim, upload(b, &b.pl_fused_g, pfg, st));
  b.n_fused_g = (int)pfg.size();
  HIPCHK(errsim, upload(b, &b.pl_fused_ng, pfng, st));
  b.n_fused_ng = (int)pfng.size();
  HIPCHK(errsim, upload(b, &b.wl_sph, wsph, st));
  b.n_big_blk = (int)wbig.size();
  if (!wbig.empty()) HIPCHK(errsim, upload(b, &b.wl_big, wbig, st));
  for (int l = 0; l <= 10; ++l) {
    b.n_tree[l] = (int)wtree[l].size();
    b.wl_tree[l] = nullptr;
    if (!wtree[l].empty()) HIPCHK(errsim, upload(b, &b.wl_tree[l], wtree[l], st));
  }
  for (int g = 0; g < 3; ++g) {
    HIPCHK(errsim, upload(b, &b.gl[g], glg[g], st));
    b.n_grav[g] = (int)glg[g].size();
    // largest items first: the blocks are handed out in launch order, so
    // the launch ends on the smallest ones
    std::stable_sort(gmw[g].begin(), gmw[g].end(),
                     [](const auto& a, const auto& c) { return a.first > c.first; });
    for (const auto& e : gmw[g]) gmg[g].push_back(e.second);
    HIPCHK(errsim, upload(b, &b.gm[g], gmg[g], st));
    b.n_gmulti[g] = (int)gmg[g].size();
    HIPCHK(errsim, upload(b, &b.gs[g], gsg[g], st));
    b.n_gsplit[g] = (int)gsg[g].size();
    b.grav_tile[g] = tiles[g];
  }
  b.n_grav_groups = n_groups;
  HIPCHK(errsim, upload(b, &b.seg_cells, sc, st));
  HIPCHK(errsim, upload(b, &b.item_cells, ic, st));
  HIPCHK(errsim, upload(b, &b.seg_pairs, sp, st));
  HIPCHK(errsim, upload(b, &b.item_pairs, ip, st));
  std::vector<uint32_t> zc(std::max<size_t>(ic.size(), 1), 0u), zp(std::max<size_t>(ip.size(), 1), 0u);
  HIPCHK(errsim, upload(b, &b.sums_cells, zc, st));
  HIPCHK(errsim, upload(b, &b.sums_pairs, zp, st));
  b.n_agg_blk = (int)wa.size();
  b.reduce_stage = tot_na >= kReduceStageMin;
  b.n_sph_blk = (int)wsph.size();
  b.max_items_cells = b.max_items_pairs = 0;
  for (const ScanSeg& g : sc) b.max_items_cells = std::max(b.max_items_cells, (int)g.n_items);
  for (const ScanSeg& g : sp) b.max_items_pairs = std::max(b.max_items_pairs, (int)g.n_items);
  b.n_seg_cells = (int)sc.size();
  b.n_item_cells = (int)ic.size();
  b.n_seg_pairs = (int)sp.size();
  b.n_item_pairs = (int)ip.size();
  b.dirty = false;
  return DEM_OK;
}

// Kernel families of one step, in launch order (profiling names).
constexpr int kNumStages = 16;
constexpr int kStageGravity = 11;
constexpr int kStageFusedA = 14;           // k_fused parts 1 and 3
constexpr int kStageFusedB = 15;           // k_fused part 2
const char* const kStageNames =
    "integrate;reconstruct;grid;bin;scan_cells;scatter;cell_sort;search_count;"
    "scan_pairs;search_write;forces;gravity;reduce;finish;fused_a;fused_b";

// Second stream and fork/join events of a batch (default priority).
hipError_t ensure_side(Batch& b) {
  hipError_t e = hipSuccess;
  if (!b.side) e = hipStreamCreateWithFlags(&b.side, hipStreamNonBlocking);
  if (e == hipSuccess && !b.fork_ev) e = hipEventCreateWithFlags(&b.fork_ev, hipEventDisableTiming);
  if (e == hipSuccess && !b.join_ev) e = hipEventCreateWithFlags(&b.join_ev, hipEventDisableTiming);
  return e;
}

void release_side(Batch& b) {
  if (b.side) (void)hipStreamDestroy(b.side);
  if (b.fork_ev) (void)hipEventDestroy(b.fork_ev);
  if (b.join_ev) (void)hipEventDestroy(b.join_ev);
  b.side = nullptr;
  b.fork_ev = b.join_ev = nullptr;
}

// Enqueue one pass of the step (mode kModeStep or kModeInit) for a batch.
// mark(k, stream, begin) is called before (begin) and after each stage k on
// the stream that runs it.  Gravity depends only on the sorted copies of the
// cell sort and is read only by the member reduction, so with `overlap` it runs on the
// batch's second stream beside the search, scan and force kernels (the
// captured step); without, every stage runs in order on one stream (the
// t0 evaluation, the stateless hooks, and the profiled passes, whose event
// spans then time each stage alone).
template <typename Mark>
void enqueue_pass_marked(Batch& b, hipStream_t st, int mode, Mark mark, bool overlap) {
  const int np = (int)b.members.size();
  const bool staged = b.n_staged > 0;
  auto stage = [&](int k, hipStream_t s, bool run, auto&& launch) {
    mark(k, s, true);
    if (run) launch(s);
    mark(k, s, false);
  };
  // small piles: their whole step (part 3), or the stages before gravity (part 1)
  stage(kStageFusedA, st, b.n_fused_ng + b.n_fused_g > 0, [&](hipStream_t s) {
    launch_fused(s, b.d_table, b.pl_fused_ng, b.n_fused_ng, b.cp, mode, 3, b.precision);
    launch_fused(s, b.d_table, b.pl_fused_g, b.n_fused_g, b.cp, mode, 1, b.precision);
  });
  stage(0, st, staged, [&](hipStream_t s) {
    launch_integrate(s, b.d_table, b.wl_agg, b.n_agg_blk, b.cp, mode);
  });
  stage(1, st, staged, [&](hipStream_t s) {
    launch_reconstruct(s, b.d_table, b.wl_sph, b.n_sph_blk);
  });
  stage(2, st, staged, [&](hipStream_t s) { launch_grid(s, b.d_table, np, mode, b.cp.dt); });
  stage(3, st, staged, [&](hipStream_t s) { launch_bin(s, b.d_table, b.wl_sph, b.n_sph_blk); });
  stage(4, st, staged, [&](hipStream_t s) {
    launch_scan(s, b.seg_cells, b.n_seg_cells, b.item_cells, b.n_item_cells, b.sums_cells,
                b.max_items_cells);
  });
  stage(5, st, staged, [&](hipStream_t s) {
    launch_scatter(s, b.d_table, b.wl_sph, b.n_sph_blk);
  });
  stage(6, st, staged, [&](hipStream_t s) {
    launch_cell_sort(s, b.d_table, b.wl_sph, b.n_sph_blk);
  });
  const bool fork = overlap && b.any_grav && b.side && staged;
  auto gravity = [&](hipStream_t s) {
    launch_gravity_records(s, b.d_table, b.wl_grav, b.n_grav_blk, b.precision);
    for (int g = 0; g < b.n_grav_groups; ++g) {
      launch_gravity_tiles(s, b.d_table, b.gl[g], b.n_grav[g], b.precision, b.all_soft,
                           b.grav_tile[g], false);
      launch_gravity_tiles(s, b.d_table, b.gm[g], b.n_gmulti[g], b.precision, b.all_soft,
                           b.grav_tile[g], true);
      launch_gravity_split(s, b.d_table, b.gs[g], b.n_gsplit[g], b.precision, b.all_soft,
                           b.grav_tile[g]);
    }
    if (b.any_direct) launch_gravity_combine(s, b.d_table, b.wl_grav, b.n_grav_blk, b.precision);
    if (b.any_tree) launch_tree(s, b.d_table, b.wl_tree, b.n_tree, b.tree_leaf_levels, b.wl_sph,
                               b.n_sph_blk, b.tree_order);
  };
  if (fork) {
    (void)hipEventRecord(b.fork_ev, st);
    (void)hipStreamWaitEvent(b.side, b.fork_ev, 0);
    stage(kStageGravity, b.side, true, gravity);
    (void)hipEventRecord(b.join_ev, b.side);
  }
  stage(7, st, staged, [&](hipStream_t s) {
    launch_search(s, b.d_table, b.wl_sph, b.n_sph_blk, 0);
    if (b.n_big_blk) launch_search_big(s, b.d_table, b.wl_big, b.n_big_blk, 0);
  });
  stage(8, st, staged, [&](hipStream_t s) {
    launch_scan(s, b.seg_pairs, b.n_seg_pairs, b.item_pairs, b.n_item_pairs, b.sums_pairs,
                b.max_items_pairs);
  });
  stage(9, st, staged, [&](hipStream_t s) {
    launch_search(s, b.d_table, b.wl_sph, b.n_sph_blk, 1);
    if (b.n_big_blk) launch_search_big(s, b.d_table, b.wl_big, b.n_big_blk, 1);
  });
  stage(10, st, staged, [&](hipStream_t s) {
    launch_forces(s, b.d_table, b.wl_sph, b.n_sph_blk, b.cp, b.precision);
  });
  if (fork) (void)hipStreamWaitEvent(st, b.join_ev, 0);
  else stage(kStageGravity, st, b.any_grav, gravity);
  stage(kStageFusedB, st, b.n_fused_g > 0, [&](hipStream_t s) {
    launch_fused(s, b.d_table, b.pl_fused_g, b.n_fused_g, b.cp, mode, 2, b.precision);
  });
  stage(12, st, staged, [&](hipStream_t s) {
    launch_reduce(s, b.d_table, b.wl_agg, b.n_agg_blk, b.cp, mode, b.reduce_stage);
  });
  stage(13, st, staged, [&](hipStream_t s) { launch_finish(s, b.d_table, np, mode, b.cp.dt); });
}

void enqueue_pass(Batch& b, hipStream_t st, int mode, bool overlap = false) {
  enqueue_pass_marked(b, st, mode, [](int, hipStream_t, bool) {}, overlap);
}

dem_status ensure_graph(Batch& b, hipStream_t st, dem_sim* errsim) {
  if (b.graph) return DEM_OK;
  HIPCHK(errsim, ensure_side(b));
  hipStream_t cap = st;
  bool own_stream = false;
  if (cap == nullptr) {
    // capture needs a non-null stream
    HIPCHK(errsim, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    own_stream = true;
  }
  HIPCHK(errsim, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  enqueue_pass(b, cap, kModeStep, true);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cap, &g);
  if (own_stream) (void)hipStreamDestroy(cap);
  if (e != hipSuccess) return fail(errsim, DEM_ERR_DEVICE, hip_msg(e, "graph capture"));
  b.graph_def = g;
  HIPCHK(errsim, hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0));
  return DEM_OK;
}

// Eager launches of n_steps passes with a HIP event between consecutive
// kernels on the stream; accumulates each kernel family's milliseconds.
dem_status profiled_passes(Batch& b, hipStream_t st, int64_t n_steps,
                           std::vector<hipEvent_t>& events, std::vector<double>& prof_ms,
                           int64_t& prof_steps, dem_sim* errsim) {
  const size_t per_step = size_t(2) * kNumStages;
  const size_t need = size_t(n_steps) * per_step;
  while (events.size() < need) {
    hipEvent_t ev;
    HIPCHK(errsim, hipEventCreate(&ev));
    events.push_back(ev);
  }
  hipError_t rec = hipSuccess;
  for (int64_t k = 0; k < n_steps; ++k) {
    hipEvent_t* ev = &events[size_t(k) * per_step];
    enqueue_pass_marked(b, st, kModeStep, [&](int m, hipStream_t s, bool begin) {
      if (rec == hipSuccess) rec = hipEventRecord(ev[2 * m + (begin ? 0 : 1)], s);
    }, false);
  }
  HIPCHK(errsim, rec);
  HIPCHK(errsim, hipStreamSynchronize(st));
  prof_ms.resize(kNumStages, 0.0);
  for (int64_t k = 0; k < n_steps; ++k) {
    hipEvent_t* ev = &events[size_t(k) * per_step];
    for (int m = 0; m < kNumStages; ++m) {
      float ms = 0.f;
      HIPCHK(errsim, hipEventElapsedTime(&ms, ev[2 * m], ev[2 * m + 1]));
      prof_ms[m] += ms;
    }
  }
  prof_steps += n_steps;
  return DEM_OK;
}

// Eager launches of n_steps passes as the step graph orders them (gravity on
// the second stream beside the contact kernels), with a HIP event before and
// after the gravity stage only, on the stream that runs it; accumulates the
// gravity stage's milliseconds.
dem_status gravity_timed_passes(Batch& b, hipStream_t st, int64_t n_steps,
                                std::vector<hipEvent_t>& events, std::vector<double>& prof_ms,
                                int64_t& prof_steps, dem_sim* errsim) {
  HIPCHK(errsim, ensure_side(b));
  const size_t need = size_t(2) * n_steps;
  while (events.size() < need) {
    hipEvent_t ev;
    HIPCHK(errsim, hipEventCreate(&ev));
    events.push_back(ev);
  }
  hipError_t rec = hipSuccess;
  for (int64_t k = 0; k < n_steps; ++k) {
    hipEvent_t* ev = &events[size_t(2) * k];
    enqueue_pass_marked(b, st, kModeStep, [&](int m, hipStream_t s, bool begin) {
      if (m == kStageGravity && rec == hipSuccess) rec = hipEventRecord(ev[begin ? 0 : 1], s);
    }, true);
  }
  HIPCHK(errsim, rec);
  HIPCHK(errsim, hipStreamSynchronize(st));
  prof_ms.resize(kNumStages, 0.0);
  for (int64_t k = 0; k < n_steps; ++k) {
    float ms = 0.f;
    HIPCHK(errsim, hipEventElapsedTime(&ms, events[size_t(2) * k], events[size_t(2) * k + 1]));
    prof_ms[kStageGravity] += ms;
  }
  prof_steps += n_steps;
  return DEM_OK;
}

dem_status valid_params(const dem_params* p, std::string* why) {
  auto bad = [&](const char* m) {
    *why = m;
    return DEM_ERR_INVALID_ARG;
  };
  if (!p) return bad("params is NULL");
  const double vals[] = {p->dt, p->G, p->softening_frac, p->k_n, p->k_t, p->eps_n, p->eps_t,
                         p->mu_s, p->mu_r, p->mu_t, p->k_r, p->k_q};
  for (double v : vals)
    if (!std::isfinite(v)) return bad("non-finite parameter");
  if (!(p->dt > 0)) return bad("dt must be > 0");
  if (p->G < 0 || p->softening_frac < 0) return bad("G and softening_frac must be >= 0");
  if (!(p->k_n > 0) || !(p->k_t > 0)) return bad("spring constants must be > 0");
  if (!(p->eps_n > 0 && p->eps_n <= 1) || !(p->eps_t > 0 && p->eps_t <= 1))
    return bad("restitution coefficients must be in (0, 1]");
  if (p->mu_s < 0 || p->mu_r < 0 || p->mu_t < 0) return bad("friction coefficients must be >= 0");
  if (p->periodic) {
    if (!(p->box[0] > 0) || p->box[1] != p->box[0] || p->box[2] != p->box[0])
      return bad("periodic box must be a cube with positive side");
  }
  if (p->precision != DEM_PREC_FP64 && p->precision != DEM_PREC_FP32_FORCE)
    return bad("unknown precision");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(p->g[k])) return bad("non-finite uniform field");
  if (p->n_walls < 0 || p->n_walls > 6) return bad("n_walls must be in 0..6");
  if (p->n_walls > 0 && p->periodic) return bad("walls need an open (non-periodic) system");
  if (!std::isfinite(p->shake_omega) || !std::isfinite(p->shake_phase))
    return bad("non-finite shaking frequency or phase");
  if (p->gravity_tree) {
    if (p->periodic) return bad("tree gravity needs an open (non-periodic) system");
    if (!(p->tree_theta > 0.0 && p->tree_theta <= 1.0)) return bad("tree_theta must be in (0, 1]");
    if (p->tree_leaf < 1 || p->tree_leaf > 4096) return bad("tree_leaf must be in 1..4096");
    if (p->tree_order != 2 && p->tree_order != 4) return bad("tree_order must be 2 or 4");
  }
  for (int w = 0; w < p->n_walls; ++w) {
    double nn = 0.0;
    for (int k = 0; k < 4; ++k)
      if (!std::isfinite(p->walls[w][k])) return bad("non-finite wall");
    for (int k = 0; k < 3; ++k) {
      if (!std::isfinite(p->shake_amp[w][k])) return bad("non-finite shaking amplitude");
      nn += p->walls[w][k] * p->walls[w][k];
    }
    if (!(std::fabs(std::sqrt(nn) - 1.0) <= 1e-12)) return bad("wall normal must be a unit vector");
  }
  return DEM_OK;
}

ContactParams contact_params(const dem_params& p) {
  ContactParams cp{};
  cp.dt = p.dt;
  cp.k_n = p.k_n;
  cp.k_t = p.k_t;
  cp.k_r = p.k_r < 0 ? p.k_t : p.k_r;
  cp.k_q = p.k_q < 0 ? p.k_t : p.k_q;
  cp.mu_s = p.mu_s;
  cp.mu_r = p.mu_r;
  cp.mu_t = p.mu_t;
  cp.damp_n = dashpot_factor(p.eps_n);
  cp.damp_t = dashpot_factor(p.eps_t);
  cp.max_overlap_frac = p.max_overlap_frac;
  return cp;
}

void release_pile(dem_sim* s) {
  for (void* p : s->bufs) s->alloc.release(p);
  s->bufs.clear();
  s->bytes = 0;
}

dem_status alloc_pile(dem_sim* s, int64_t na, int64_t ns) {
  PileDev h{};
  s->sz = pile_sizes(s->prm, na, ns, s->c_max, s->tune.gravity_tile, s->tune.gravity_form);
  BufList L;
  plan_pile(h, s->sz, L);
  for (auto& r : L.req) {
    void* p = s->alloc.alloc(r.second);
    if (!p) {
      release_pile(s);
      return fail(s, DEM_ERR_OOM, "device allocation failed");
    }
    s->bufs.push_back(p);
    s->bytes += r.second;
    *r.first = p;
  }
  h.na = (int32_t)na;
  h.ns = (int32_t)ns;
  h.cap_pairs = (int32_t)s->sz.cap;
  h.bits = choose_bits(ns);
  h.periodic = s->prm.periodic ? 1 : 0;
  h.member_scan = s->tune.member_scan;
  h.member_read = s->tune.member_read;
  h.g_tile = (int32_t)s->sz.g_tile;
  h.g_nt = (int32_t)s->sz.g_nt;
  h.g_form = s->sz.g_form;
  h.g_np = (int32_t)s->sz.g_np;
  h.n_rblk = (int32_t)s->sz.n_rblk;
  h.box = s->prm.box[0];
  h.G = s->prm.G;
  h.soft_frac = s->prm.softening_frac;
  h.spin_dw = s->forcing.spin_dw;
  h.stop_growth = s->forcing.stop_growth;
  h.R0 = 0.0;
  h.tree = s->sz.tree ? 1 : 0;
  h.tree_leaf = s->prm.tree_leaf;
  h.theta = s->prm.tree_theta;
  h.tree_order = s->prm.tree_order;
  h.n_walls = s->prm.n_walls;
  for (int k = 0; k < 3; ++k) h.gfield[k] = s->prm.g[k];
  for (int w = 0; w < 6; ++w) {
    for (int k = 0; k < 4; ++k) h.wall[w][k] = w < h.n_walls ? s->prm.walls[w][k] : 0.0;
    for (int k = 0; k < 3; ++k) h.wall_amp[w][k] = w < h.n_walls ? s->prm.shake_amp[w][k] : 0.0;
  }
  h.wall_omega = s->prm.shake_omega;
  h.wall_phase = s->prm.shake_phase;
  h.pert_on = s->forcing.pert_mass > 0.0 ? 1 : 0;
  h.pert_M = s->forcing.pert_mass;
  for (int k = 0; k < 3; ++k) {
    for (int q = 0; q < 2; ++q) {
      h.pert_r[q][k] = s->forcing.pert_pos[k];
      h.pert_v[q][k] = s->forcing.pert_vel[k];
      h.pert_a[q][k] = 0.0;
    }
  }
  h.s_cut = INFINITY;
  h.s_small = 0.0;
  h.n_big = 0;
  h.parity = 0;
  h.status = 0;
  h.step = 0;
  h.fail_step = -1;
  s->h = h;
  return DEM_OK;
}

// Upload the host mirror into a batch table slot.
hipError_t put_entry(const dem_sim* s, PileDev* dst, hipStream_t st) {
  return hipMemcpyAsync(dst, &s->h, sizeof(PileDev), hipMemcpyHostToDevice, st);
}

// Fields of a table entry that the kernels update (everything else is set
// by the host): bookkeeping and the perturber's state.
void copy_device_fields(PileDev& dst, const PileDev& src) {
  dst.parity = src.parity;
  dst.status = src.status;
  dst.step = src.step;
  dst.fail_step = src.fail_step;
  dst.n_pairs = src.n_pairs;
  dst.R0 = src.R0;
  for (int q = 0; q < 2; ++q)
    for (int k = 0; k < 3; ++k) {
      dst.pert_r[q][k] = src.pert_r[q][k];
      dst.pert_v[q][k] = src.pert_v[q][k];
      dst.pert_a[q][k] = src.pert_a[q][k];
    }
}

// Read back a table entry into the host mirror (after the stream is idle).
hipError_t get_entry(dem_sim* s, const PileDev* src, hipStream_t st) {
  PileDev tmp;
  hipError_t e = hipMemcpyAsync(&tmp, src, sizeof(PileDev), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  copy_device_fields(s->h, tmp);
  return hipSuccess;
}

const PileDev* entry_of(const dem_sim* s) {
  if (s->engine) return s->engine->batch.d_table + s->engine_slot;
  return s->own.d_table;
}

hipStream_t stream_of(const dem_sim* s) { return s->engine ? s->engine->stream : s->stream; }

dem_status status_code(int st) {
  if (st & kStCapacity) return DEM_ERR_CAPACITY;
  if (st & kStUnstable) return DEM_ERR_UNSTABLE;
  if (st & kStStopped) return DEM_STOPPED;
  return DEM_OK;
}

// Whether a system runs its whole step in one workgroup (k_fused): never
// with tree gravity; else as tuned, or automatically for small systems.
int fused_choice(const dem_sim* s, int64_t ns) {
  if ((s->prm.gravity_tree && s->prm.G != 0.0) || s->tune.fused == 2) return 0;
  if (s->tune.fused == 1) return 1;
  return ns <= kFusedAutoMax ? 1 : 0;
}

dem_status ensure_own_table(dem_sim* s) {
  Batch& b = s->own;
  if (!b.d_table) {
    HIPCHK(s, hipMalloc(&b.d_table, sizeof(PileDev)));
    b.table_cap = 1;
  }
  b.members.assign(1, s);
  b.cp = contact_params(s->prm);
  b.precision = s->prm.precision;
  return DEM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// allocation-free contact search: every scratch buffer in one static array
// ---------------------------------------------------------------------------

namespace {

constexpr int64_t kNoAllocMaxSpheres = 65536;
constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 20;
constexpr size_t kNoAllocScratchBytes = size_t(40) << 20;
constexpr int kMaxDevices = 64;

}  // namespace

// Scratch of dem_find_contacts_noalloc: one copy per GPU, held until the
// process ends.  In host code this name is only a stand-in for the symbol;
// the device address comes from hipGetSymbolAddress (noalloc_scratch()).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

// First bytes of the scratch: the largest radius (bit pattern of a positive
// double, ordered like an unsigned integer) and a flag for invalid input.
struct NoAllocHdr {
  unsigned long long max_r_bits;
  uint32_t bad;
  uint32_t pad;
};

// One thread per sphere: row-major device positions into the search's
// component-major array; radius and position checks; largest radius.
__global__ __launch_bounds__(kBlock) void k_noalloc_ingest(const double* __restrict__ pos,
                                                           const double* __restrict__ rad, int n,
                                                           double* __restrict__ r,
                                                           NoAllocHdr* __restrict__ hdr) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double smax = 0.0;
  bool bad = false;
  if (i < n) {
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2], s = rad[i];
    r[i] = x;
    r[n + i] = y;
    r[2 * n + i] = z;
    bad = !(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(s) && s > 0.0);
    smax = bad ? 0.0 : s;
  }
  for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off));
  const bool any_bad = __any(bad);
  if ((threadIdx.x & 63) == 0) {
    if (any_bad) atomicOr(&hdr->bad, 1u);
    if (smax > 0.0) atomicMax(&hdr->max_r_bits, (unsigned long long)__double_as_longlong(smax));
  }
}

// One thread per sphere: its upper run as canonical keys, up to cap in all.
__global__ __launch_bounds__(kBlock) void k_noalloc_keys(const uint32_t* __restrict__ off,
                                                         const uint32_t* __restrict__ pj, int n,
                                                         uint64_t* __restrict__ out, int64_t cap) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  for (int64_t p = off[i], p1 = off[i + 1]; p < p1 && p < cap; ++p)
    out[p] = (uint64_t(i) << 32) | pj[p];
}

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device,
// with that device current).
hipError_t noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Bump placement inside the scratch (256-byte aligned pieces).
struct Placer {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(int64_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += round256(size_t(std::max<int64_t>(count, 1)) * sizeof(T));
    return p;
  }
};

// Places the header, the table entry, the work lists and every buffer the
// search kernels touch for n spheres; returns the bytes used.
struct NoAllocPlan {
  NoAllocHdr* hdr;
  PileDev* entry;
  WorkItem* wl;
  ScanSeg* seg_cells;
  ScanItem* item_cells;
  uint32_t* sums_cells;
  ScanSeg* seg_pairs;
  ScanItem* item_pairs;
  uint32_t* sums_pairs;
  int n_blk, n_item_cells, n_item_pairs, max_items_cells, max_items_pairs;
  int64_t cells;
  size_t bytes;
};

int64_t scan_items(int64_t n) { return (n + kScanChunk - 1) / kScanChunk; }

NoAllocPlan plan_noalloc(char* base, int64_t n, PileDev& h) {
  Placer L{base};
  NoAllocPlan q{};
  q.cells = int64_t(1) << (3 * choose_bits(n));
  q.n_blk = (int)((n + kBlock - 1) / kBlock);
  q.n_item_cells = (int)scan_items(q.cells + 1);
  q.max_items_cells = q.n_item_cells;
  q.max_items_pairs = (int)scan_items(n);
  q.n_item_pairs = 2 * q.max_items_pairs;
  q.hdr = L.take<NoAllocHdr>(1);
  q.entry = L.take<PileDev>(1);
  q.wl = L.take<WorkItem>(q.n_blk);
  q.seg_cells = L.take<ScanSeg>(1);
  q.item_cells = L.take<ScanItem>(q.n_item_cells);
  q.sums_cells = L.take<uint32_t>(q.n_item_cells);
  q.seg_pairs = L.take<ScanSeg>(2);
  q.item_pairs = L.take<ScanItem>(q.n_item_pairs);
  q.sums_pairs = L.take<uint32_t>(q.n_item_pairs);
  h.r = L.take<double>(3 * n);
  h.key = L.take<uint32_t>(n);
  h.sidx = L.take<uint32_t>(n);
  h.sidx_raw = L.take<uint32_t>(n);
  h.slot = L.take<uint32_t>(n);
  h.xs = L.take<double>(4 * n);
  h.xg = L.take<SortedGeom>(n);
  h.sid = L.take<SortedId>(n);
  h.bpart = L.take<double>(kBbox * q.n_blk);
  h.grid = L.take<Grid>(1);
  h.cell_cnt = L.take<uint32_t>(q.cells + 1);
  h.cell_start = L.take<uint32_t>(q.cells + 2);
  h.run_cache = L.take<uint32_t>(2 * kRunCache * n);
  h.cnt_up = L.take<uint32_t>(n);
  h.cnt_lo = L.take<uint32_t>(n);
  h.up_off[0] = L.take<uint32_t>(n + 1);
  h.up_off[1] = L.take<uint32_t>(n + 1);
  h.lo_off = L.take<uint32_t>(n + 1);
  h.pair_j[0] = L.take<uint32_t>(kNoAllocMaxPairs);
  h.pair_j[1] = L.take<uint32_t>(kNoAllocMaxPairs);
  h.lo_nbr = L.take<uint32_t>(kNoAllocMaxPairs);
  q.bytes = L.off;
  return q;
}

}  // namespace

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* dem_last_error(const dem_sim* sim) {
  if (sim) return sim->err.c_str();
  return g_error.c_str();
}

size_t dem_footprint_bytes(const dem_params* params, int64_t n_agg, int64_t n_sph) {
  if (!params || n_agg <= 0 || n_sph <= 0) return 0;
  int c = params->max_contacts_per_sphere > 0 ? params->max_contacts_per_sphere : kDefaultContacts;
  PileDev h{};
  BufList L;
  plan_pile(h, pile_sizes(*params, n_agg, n_sph, c, 0), L);
  return L.total();
}

dem_status dem_create(const dem_params* params, const dem_allocator* alloc, void* hip_stream,
                      dem_sim** out) {
  if (!out) return fail(nullptr, DEM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  std::string why;
  if (valid_params(params, &why) != DEM_OK) return fail(nullptr, DEM_ERR_INVALID_ARG, why);
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(nullptr, DEM_ERR_INVALID_ARG, "allocator needs alloc and free");
  dem_sim* s = new dem_sim();
  s->prm = *params;
  if (alloc) {
    s->alloc.user = *alloc;
    s->alloc.has_user = true;
  }
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->c_max = params->max_contacts_per_sphere > 0 ? params->max_contacts_per_sphere : kDefaultContacts;
  *out = s;
  return DEM_OK;
}

dem_status dem_destroy(dem_sim* s) {
  if (!s) return DEM_OK;
  if (s->engine) dem_engine_detach(s->engine, s);
  (void)hipStreamSynchronize(s->stream);
  for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
  free_meta(s->own);
  release_side(s->own);
  if (s->own.d_table) (void)hipFree(s->own.d_table);
  release_pile(s);
  delete s;
  return DEM_OK;
}

dem_status dem_add_aggregates(dem_sim* s, int64_t n_agg, const int32_t* spa, const double* pos,
                              const double* radius, const double* mass, const double* agg_vel,
                              const double* agg_spin, int64_t* first_agg_id) {
  if (!s) return fail(nullptr, DEM_ERR_INVALID_ARG, "sim is NULL");
  if (s->has_aggs || s->stepped) return fail(s, DEM_ERR_STATE, "aggregates already added");
  if (s->engine) return fail(s, DEM_ERR_STATE, "system is attached to an engine");
  if (n_agg <= 0 || !spa || !pos || !radius || !mass)
    return fail(s, DEM_ERR_INVALID_ARG, "empty input or NULL array");
  int64_t ns = 0;
  for (int64_t a = 0; a < n_agg; ++a) {
    if (spa[a] <= 0) return fail(s, DEM_ERR_INVALID_ARG, "aggregate with no spheres");
    ns += spa[a];
  }
  if (ns > (int64_t(1) << 30)) return fail(s, DEM_ERR_INVALID_ARG, "too many spheres");
  double smax = 0.0;
  for (int64_t i = 0; i < ns; ++i) {
    if (!std::isfinite(radius[i]) || !std::isfinite(mass[i]) || radius[i] <= 0 || mass[i] <= 0)
      return fail(s, DEM_ERR_INVALID_ARG, "radius and mass must be finite and > 0");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(pos[3 * i + k])) return fail(s, DEM_ERR_INVALID_ARG, "non-finite position");
    smax = std::max(smax, radius[i]);
  }
  for (int64_t k = 0; k < 3 * n_agg; ++k) {
    if (agg_vel && !std::isfinite(agg_vel[k])) return fail(s, DEM_ERR_INVALID_ARG, "non-finite velocity");
    if (agg_spin && !std::isfinite(agg_spin[k])) return fail(s, DEM_ERR_INVALID_ARG, "non-finite spin");
  }
  if (require_device(s) != DEM_OK) return DEM_ERR_DEVICE;
  double s_cut, s_small;
  int n_big;
  split_big(radius, ns, &s_cut, &s_small, &n_big);
  if (s->prm.gravity_tree && s->prm.G != 0.0) {   // the tree covers every sphere
    s_cut = INFINITY;
    s_small = smax;
    n_big = 0;
  }
  const double cell_min = s->tune.cell_scale * 2.0 * s_small;
  dem_status st = alloc_pile(s, n_agg, ns);
  if (st != DEM_OK) return st;
  s->h.fused = fused_choice(s, ns);
  s->h.cell_min = cell_min;
  s->h.s_cut = s_cut;
  s->h.s_small = s_small;
  s->h.n_big = n_big;
  if (s->prm.periodic) s->h.n_periodic = periodic_cells(s->prm.box[0], cell_min, s->h.bits);
  hipStream_t str = s->stream;
  // constants: membership, radius, mass
  std::vector<int32_t> first(n_agg), agg(ns);
  int64_t off = 0;
  for (int64_t a = 0; a < n_agg; ++a) {
    first[a] = (int32_t)off;
    for (int64_t k = 0; k < spa[a]; ++k) agg[off + k] = (int32_t)a;
    off += spa[a];
  }
  HIPCHK(s, hipMemcpyAsync(s->h.first, first.data(), n_agg * 4, hipMemcpyHostToDevice, str));
  HIPCHK(s, hipMemcpyAsync(s->h.count, spa, n_agg * 4, hipMemcpyHostToDevice, str));
  HIPCHK(s, hipMemcpyAsync(s->h.agg, agg.data(), ns * 4, hipMemcpyHostToDevice, str));
  HIPCHK(s, hipMemcpyAsync(s->h.s, radius, ns * 8, hipMemcpyHostToDevice, str));
  HIPCHK(s, hipMemcpyAsync(s->h.m, mass, ns * 8, hipMemcpyHostToDevice, str));
  // staging for the set-up kernel
  double *d_pos = nullptr, *d_vel = nullptr, *d_spin = nullptr;
  HIPCHK(s, hipMalloc(&d_pos, ns * 24));
  HIPCHK(s, hipMemcpyAsync(d_pos, pos, ns * 24, hipMemcpyHostToDevice, str));
  if (agg_vel) {
    HIPCHK(s, hipMalloc(&d_vel, n_agg * 24));
    HIPCHK(s, hipMemcpyAsync(d_vel, agg_vel, n_agg * 24, hipMemcpyHostToDevice, str));
  }
  if (agg_spin) {
    HIPCHK(s, hipMalloc(&d_spin, n_agg * 24));
    HIPCHK(s, hipMemcpyAsync(d_spin, agg_spin, n_agg * 24, hipMemcpyHostToDevice, str));
  }
  // zero the contact lists (empty history) and cell counts
  launch_fill_u32(str, s->h.up_off[0], 0u, ns + 1);
  launch_fill_u32(str, s->h.up_off[1], 0u, ns + 1);
  launch_fill_u32(str, s->h.lo_off, 0u, ns + 1);
  launch_fill_u32(str, s->h.cell_cnt, 0u, s->sz.cells + 1);
  st = ensure_own_table(s);
  if (st != DEM_OK) return st;
  HIPCHK(s, put_entry(s, s->own.d_table, str));
  st = rebuild(s->own, str, s);
  if (st != DEM_OK) return st;
  launch_setup(str, s->own.d_table, s->own.wl_agg_all, s->own.n_agg_all_blk, d_pos, d_vel,
               d_spin);
  // initial evaluation at t0 (forces, torques and accelerations)
  enqueue_pass(s->own, str, kModeInit);
  HIPCHK(s, hipGetLastError());
  HIPCHK(s, get_entry(s, s->own.d_table, str));
  (void)hipFree(d_pos);
  if (d_vel) (void)hipFree(d_vel);
  if (d_spin) (void)hipFree(d_spin);
  s->has_aggs = true;
  if (first_agg_id) *first_agg_id = 0;
  if (s->h.status != 0) {
    dem_status code = status_code(s->h.status);
    return fail(s, code, code == DEM_ERR_CAPACITY ? "initial contacts exceed capacity"
                                                  : "initial state unstable");
  }
  return DEM_OK;
}

dem_status dem_step(dem_sim* s, int64_t n_steps) {
  if (!s) return fail(nullptr, DEM_ERR_INVALID_ARG, "sim is NULL");
  if (s->engine) return fail(s, DEM_ERR_STATE, "system is attached to an engine");
  if (!s->has_aggs) return fail(s, DEM_ERR_STATE, "no aggregates");
  if (n_steps < 0) return fail(s, DEM_ERR_INVALID_ARG, "negative step count");
  if (s->h.status != 0) {
    const dem_status code = status_code(s->h.status);
    if (code == DEM_STOPPED) return DEM_STOPPED;   // reset the forcing to go on
    return fail(s, code, "system has failed; restore it");
  }
  s->stepped = true;
  if (n_steps == 0) return DEM_OK;
  if (s->profiling == 1) {
    dem_status st = profiled_passes(s->own, s->stream, n_steps, s->events, s->prof_ms,
                                    s->prof_steps, s);
    if (st != DEM_OK) return st;
  } else if (s->profiling == 2) {
    dem_status st = gravity_timed_passes(s->own, s->stream, n_steps, s->events, s->prof_ms,
                                         s->prof_steps, s);
    if (st != DEM_OK) return st;
  } else {
    dem_status st = ensure_graph(s->own, s->stream, s);
    if (st != DEM_OK) return st;
    for (int64_t k = 0; k < n_steps; ++k) HIPCHK(s, hipGraphLaunch(s->own.graph, s->stream));
  }
  HIPCHK(s, get_entry(s, s->own.d_table, s->stream));
  if (s->h.status != 0) {
    dem_status code = status_code(s->h.status);
    char buf[200];
    snprintf(buf, sizeof buf, "%s at step %lld; state is that at the start of that step",
             code == DEM_ERR_CAPACITY  ? "contact capacity exceeded"
             : code == DEM_STOPPED     ? "stop rule reached (bulk radius grown)"
                                       : "unstable contact",
             (long long)s->h.fail_step);
    if (code == DEM_STOPPED) {
      s->err = buf;
      return DEM_STOPPED;
    }
    return fail(s, code, buf);
  }
  return DEM_OK;
}

dem_status dem_get_counts(const dem_sim* s, int64_t* n_agg, int64_t* n_sph, int64_t* n_pairs) {
  if (!s) return fail(nullptr, DEM_ERR_INVALID_ARG, "sim is NULL");
  if (n_agg) *n_agg = s->has_aggs ? s->h.na : 0;
  if (n_sph) *n_sph = s->has_aggs ? s->h.ns : 0;
  if (n_pairs) *n_pairs = s->has_aggs ? s->h.n_pairs : 0;
  return DEM_OK;
}

namespace {

// Copy a component-major device array [k][n] into row-major host [n][k].
dem_status fetch_rows(dem_sim* s, const double* d, int k, int64_t n, double* host, hipStream_t st) {
  std::vector<double> tmp(size_t(k) * n);
  HIPCHK(s, hipMemcpyAsync(tmp.data(), d, tmp.size() * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < k; ++c) host[i * k + c] = tmp[size_t(c) * n + i];
  return DEM_OK;
}

dem_status store_rows(dem_sim* s, double* d, int k, int64_t n, const double* host, hipStream_t st) {
  std::vector<double> tmp(size_t(k) * n);
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < k; ++c) tmp[size_t(c) * n + i] = host[i * k + c];
  HIPCHK(s, hipMemcpyAsync(d, tmp.data(), tmp.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipStreamSynchronize(st));
  return DEM_OK;
}

}  // namespace

dem_status dem_read_state(dem_sim* s, dem_state* out) {
  if (!s || !out) return fail(s, DEM_ERR_INVALID_ARG, "NULL argument");
  if (!s->has_aggs) return fail(s, DEM_ERR_STATE, "no aggregates");
  hipStream_t st = stream_of(s);
  HIPCHK(s, get_entry(s, entry_of(s), st));
  const PileDev& h = s->h;
  const int cur = h.parity;
  const int64_t na = h.na, ns = h.ns;
  dem_status r = DEM_OK;
  auto rows = [&](const double* d, int k, int64_t n, double* host) {
    if (host && r == DEM_OK) r = fetch_rows(s, d, k, n, host, st);
  };
  rows(h.rA[cur], 3, na, out->agg_pos);
  rows(h.vA[cur], 3, na, out->agg_vel);
  rows(h.aA[cur], 3, na, out->agg_acc);
  rows(h.NA[cur], 3, na, out->agg_torque);
  rows(h.q[cur], 4, na, out->agg_quat);
  rows(h.wb[cur], 3, na, out->agg_spin_body);
  rows(h.M, 1, na, out->agg_mass);
  rows(h.I, 3, na, out->agg_inertia);
  rows(h.r, 3, ns, out->sph_pos);
  rows(h.v, 3, ns, out->sph_vel);
  rows(h.F, 3, ns, out->sph_force);
  rows(h.tau, 3, ns, out->sph_torque);
  rows(h.b, 3, ns, out->sph_body);
  if (r != DEM_OK) return r;
  if (out->sph_force && h.G != 0.0) {
    // the device keeps the contact force; the gravity force is added after
    // it, in the order (and so with the rounding) of the member reduction
    std::vector<double> ga(3 * ns);
    r = fetch_rows(s, h.gacc, 3, ns, ga.data(), st);
    if (r != DEM_OK) return r;
    for (int64_t k = 0; k < 3 * ns; ++k) out->sph_force[k] += ga[k];
  }
  if (out->agg_spin) {
    // space-frame spin R(q) w_b of the current state
    std::vector<double> q(4 * na), wb(3 * na);
    r = fetch_rows(s, h.q[cur], 4, na, q.data(), st);
    if (r == DEM_OK) r = fetch_rows(s, h.wb[cur], 3, na, wb.data(), st);
    if (r != DEM_OK) return r;
    for (int64_t a = 0; a < na; ++a) {
      const double w = q[4 * a], x = q[4 * a + 1], y = q[4 * a + 2], z = q[4 * a + 3];
      const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                           2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                           2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
      const double* o = &wb[3 * a];
      for (int c = 0; c < 3; ++c)
        out->agg_spin[3 * a + c] = R[3 * c] * o[0] + R[3 * c + 1] * o[1] + R[3 * c + 2] * o[2];
    }
  }
  out->n_pairs = h.n_pairs;
  out->step = h.step;
  if (out->pair_keys || out->pair_hist) {
    const int64_t np = h.n_pairs;
    std::vector<uint32_t> off(ns + 1), pj(std::max<int64_t>(np, 1));
    HIPCHK(s, hipMemcpyAsync(off.data(), h.up_off[cur], (ns + 1) * 4, hipMemcpyDeviceToHost, st));
    if (np) HIPCHK(s, hipMemcpyAsync(pj.data(), h.pair_j[cur], np * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipStreamSynchronize(st));
    if (out->pair_keys)
      for (int64_t i = 0; i < ns; ++i)
        for (uint32_t p = off[i]; p < off[i + 1]; ++p)
          out->pair_keys[p] = (uint64_t(i) << 32) | pj[p];
    if (out->pair_hist && np) {
      std::vector<double> hh(size_t(kHist) * h.cap_pairs);
      HIPCHK(s, hipMemcpyAsync(hh.data(), h.hist[cur], hh.size() * 8, hipMemcpyDeviceToHost, st));
      HIPCHK(s, hipStreamSynchronize(st));
      for (int64_t p = 0; p < np; ++p)
        for (int c = 0; c < kHist; ++c) out->pair_hist[p * kHist + c] = hh[size_t(c) * h.cap_pairs + p];
    }
  }
  return DEM_OK;
}

dem_status dem_restore_state(dem_sim* s, const dem_state* in) {
  if (!s || !in) return fail(s, DEM_ERR_INVALID_ARG, "NULL argument");
  if (!s->has_aggs) return fail(s, DEM_ERR_STATE, "no aggregates");
  if (s->engine) return fail(s, DEM_ERR_STATE, "system is attached to an engine");
  if (!in->agg_pos || !in->agg_vel || !in->agg_acc || !in->agg_torque || !in->agg_quat ||
      !in->agg_spin_body)
    return fail(s, DEM_ERR_INVALID_ARG, "restore needs the aggregate state fields");
  if (in->n_pairs < 0 || (in->n_pairs > 0 && (!in->pair_keys || !in->pair_hist)))
    return fail(s, DEM_ERR_INVALID_ARG, "restore needs pair keys and history");
  if (in->n_pairs > s->h.cap_pairs) return fail(s, DEM_ERR_CAPACITY, "checkpoint has more contacts than capacity");
  hipStream_t st = s->stream;
  HIPCHK(s, hipStreamSynchronize(st));
  PileDev& h = s->h;
  const int cur = h.parity;
  const int64_t na = h.na, ns = h.ns, np = in->n_pairs;
  dem_status r = store_rows(s, h.rA[cur], 3, na, in->agg_pos, st);
  if (r == DEM_OK) r = store_rows(s, h.vA[cur], 3, na, in->agg_vel, st);
  if (r == DEM_OK) r = store_rows(s, h.aA[cur], 3, na, in->agg_acc, st);
  if (r == DEM_OK) r = store_rows(s, h.NA[cur], 3, na, in->agg_torque, st);
  if (r == DEM_OK) r = store_rows(s, h.q[cur], 4, na, in->agg_quat, st);
  if (r == DEM_OK) r = store_rows(s, h.wb[cur], 3, na, in->agg_spin_body, st);
  if (r != DEM_OK) return r;
  // contact list as CSR of the canonical keys
  std::vector<uint32_t> off(ns + 1, 0), pj(std::max<int64_t>(np, 1));
  for (int64_t p = 0; p < np; ++p) {
    const uint64_t key = in->pair_keys[p];
    const int64_t i = int64_t(key >> 32), j = int64_t(key & 0xffffffffu);
    // a partner is a sphere j > i or a wall ns + w (sorted after the spheres)
    if (i < 0 || i >= ns || j <= i || j >= ns + h.n_walls ||
        (p > 0 && key <= in->pair_keys[p - 1]))
      return fail(s, DEM_ERR_INVALID_ARG, "pair keys must be canonical and sorted");
    off[i + 1]++;
    pj[p] = uint32_t(j);
  }
  for (int64_t i = 0; i < ns; ++i) off[i + 1] += off[i];
  HIPCHK(s, hipMemcpyAsync(h.up_off[cur], off.data(), (ns + 1) * 4, hipMemcpyHostToDevice, st));
  if (np) {
    HIPCHK(s, hipMemcpyAsync(h.pair_j[cur], pj.data(), np * 4, hipMemcpyHostToDevice, st));
    std::vector<double> col(np);
    for (int c = 0; c < kHist; ++c) {
      for (int64_t p = 0; p < np; ++p) col[p] = in->pair_hist[p * kHist + c];
      HIPCHK(s, hipMemcpyAsync(h.hist[cur] + size_t(c) * h.cap_pairs, col.data(), np * 8,
                               hipMemcpyHostToDevice, st));
      HIPCHK(s, hipStreamSynchronize(st));
    }
  }
  launch_fill_u32(st, h.cell_cnt, 0u, s->sz.cells + 1);
  h.status = 0;
  h.fail_step = -1;
  h.step = in->step;
  h.n_pairs = uint32_t(np);
  HIPCHK(s, put_entry(s, s->own.d_table, st));
  HIPCHK(s, hipStreamSynchronize(st));
  return DEM_OK;
}

dem_status dem_set_forcing(dem_sim* s, const dem_forcing* f) {
  if (!s || !f) return fail(s, DEM_ERR_INVALID_ARG, "NULL argument");
  bool ok = std::isfinite(f->spin_dw) && std::isfinite(f->pert_mass) && f->pert_mass >= 0.0 &&
            std::isfinite(f->stop_growth) && f->stop_growth >= 0.0;
  for (int k = 0; k < 3; ++k) ok = ok && std::isfinite(f->pert_pos[k]) && std::isfinite(f->pert_vel[k]);
  if (!ok) return fail(s, DEM_ERR_INVALID_ARG, "non-finite or negative forcing");
  if (f->pert_mass > 0.0 && !(s->prm.G > 0.0))
    return fail(s, DEM_ERR_INVALID_ARG, "a perturber needs G > 0");
  s->forcing = *f;
  if (!s->has_aggs) return DEM_OK;
  hipStream_t st = stream_of(s);
  HIPCHK(s, get_entry(s, entry_of(s), st));
  PileDev& h = s->h;
  h.spin_dw = f->spin_dw;
  h.stop_growth = f->stop_growth;
  h.R0 = 0.0;                        // the next evaluation sets the reference radius
  h.status &= ~kStStopped;           // a stopped system may go on under the new rule
  if (h.status == 0) h.fail_step = -1;
  h.pert_on = f->pert_mass > 0.0 ? 1 : 0;
  h.pert_M = f->pert_mass;
  for (int k = 0; k < 3; ++k) {
    h.pert_r[h.parity][k] = f->pert_pos[k];
    h.pert_v[h.parity][k] = f->pert_vel[k];
    h.pert_a[h.parity][k] = 0.0;
  }
  HIPCHK(s, put_entry(s, const_cast<PileDev*>(entry_of(s)), st));
  HIPCHK(s, hipStreamSynchronize(st));
  return DEM_OK;
}

dem_status dem_get_forcing(dem_sim* s, dem_forcing* out) {
  if (!s || !out) return fail(s, DEM_ERR_INVALID_ARG, "NULL argument");
  *out = s->forcing;
  if (!s->has_aggs) return DEM_OK;
  hipStream_t st = stream_of(s);
  PileDev cur;
  HIPCHK(s, hipMemcpyAsync(&cur, entry_of(s), sizeof(PileDev), hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  out->spin_dw = cur.spin_dw;
  out->stop_growth = cur.stop_growth;
  out->pert_mass = cur.pert_on ? cur.pert_M : 0.0;
  for (int k = 0; k < 3; ++k) {
    out->pert_pos[k] = cur.pert_r[cur.parity][k];
    out->pert_vel[k] = cur.pert_v[cur.parity][k];
  }
  return DEM_OK;
}

dem_status dem_reserve_contacts(dem_sim* s, int32_t per_sphere) {
  if (!s || per_sphere <= 0) return fail(s, DEM_ERR_INVALID_ARG, "bad argument");
  if (s->engine) return fail(s, DEM_ERR_STATE, "system is attached to an engine");
  if (!s->has_aggs) {
    s->c_max = per_sphere;
    return DEM_OK;
  }
  if (per_sphere <= s->c_max) return DEM_OK;
  // checkpoint the state on the host, allocate a second set of buffers with
  // the larger capacity, copy the constants across and restore into it; the
  // old buffers are released only once that has succeeded, so any failure
  // leaves the system as it was
  hipStream_t st = s->stream;
  HIPCHK(s, get_entry(s, s->own.d_table, st));
  const int64_t na = s->h.na, ns = s->h.ns, np = s->h.n_pairs;
  std::vector<double> rA(3 * na), vA(3 * na), aA(3 * na), NA(3 * na), q(4 * na), wb(3 * na),
      hist(kHist * std::max<int64_t>(np, 1));
  std::vector<uint64_t> keys(std::max<int64_t>(np, 1));
  dem_state io{};
  io.agg_pos = rA.data();
  io.agg_vel = vA.data();
  io.agg_acc = aA.data();
  io.agg_torque = NA.data();
  io.agg_quat = q.data();
  io.agg_spin_body = wb.data();
  io.pair_keys = keys.data();
  io.pair_hist = hist.data();
  dem_status r = dem_read_state(s, &io);
  if (r != DEM_OK) return r;
  const PileDev old = s->h;
  const Sizes old_sz = s->sz;
  std::vector<void*> old_bufs;
  old_bufs.swap(s->bufs);
  const size_t old_bytes = s->bytes;
  const int old_c = s->c_max;
  s->bytes = 0;
  auto undo = [&](dem_status code) {
    release_pile(s);                       // the new buffers (if any)
    s->bufs.swap(old_bufs);
    s->bytes = old_bytes;
    s->sz = old_sz;
    s->h = old;
    s->c_max = old_c;
    free_meta(s->own);
    if (put_entry(s, s->own.d_table, st) == hipSuccess) (void)rebuild(s->own, st, s);
    (void)hipStreamSynchronize(st);
    return code;
  };
  s->c_max = per_sphere;
  r = alloc_pile(s, na, ns);
  if (r != DEM_OK) {
    const std::string why = s->err;
    undo(r);
    return fail(s, r, why);
  }
  PileDev& h = s->h;
  h.fused = old.fused;
  h.cell_min = old.cell_min;
  h.s_cut = old.s_cut;
  h.s_small = old.s_small;
  h.n_big = old.n_big;
  h.n_periodic = old.n_periodic;
  h.step = old.step;
  for (int k = 0; k < 3; ++k) {   // the perturber continues where it was
    h.pert_r[0][k] = old.pert_r[old.parity][k];
    h.pert_v[0][k] = old.pert_v[old.parity][k];
    h.pert_a[0][k] = old.pert_a[old.parity][k];
  }
  // constants that survive, device to device
  hipError_t e = hipSuccess;
  auto copy = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
  };
  copy(h.first, old.first, na * 4);
  copy(h.count, old.count, na * 4);
  copy(h.agg, old.agg, ns * 4);
  copy(h.M, old.M, na * 8);
  copy(h.I, old.I, 3 * na * 8);
  copy(h.b, old.b, 3 * ns * 8);
  copy(h.s, old.s, ns * 8);
  copy(h.m, old.m, ns * 8);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(s, undo(DEM_ERR_DEVICE), hip_msg(e, "reserve copy"));
  launch_fill_u32(st, h.up_off[0], 0u, ns + 1);
  launch_fill_u32(st, h.up_off[1], 0u, ns + 1);
  launch_fill_u32(st, h.lo_off, 0u, ns + 1);
  free_meta(s->own);
  e = put_entry(s, s->own.d_table, st);
  if (e != hipSuccess) return fail(s, undo(DEM_ERR_DEVICE), hip_msg(e, "reserve table"));
  r = rebuild(s->own, st, s);
  if (r == DEM_OK) {
    io.n_pairs = np;
    io.step = old.step;
    r = dem_restore_state(s, &io);
  }
  if (r != DEM_OK) {
    const std::string why = s->err;
    undo(r);
    return fail(s, r, why);
  }
  // the new buffers hold the state: release the old ones
  for (void* p : old_bufs) s->alloc.release(p);
  return DEM_OK;
}

dem_status dem_set_tuning(dem_sim* s, const dem_tuning* t) {
  if (!s || !t) return fail(s, DEM_ERR_INVALID_ARG, "NULL argument");
  if (s->has_aggs) return fail(s, DEM_ERR_STATE, "tuning must be set before adding aggregates");
  if (t->gravity_tile != 0 && !tile_supported(s->prm.precision, t->gravity_tile))
    return fail(s, DEM_ERR_INVALID_ARG, "unsupported gravity tile size");
  if (!(t->cell_scale >= 1.0) || !std::isfinite(t->cell_scale))
    return fail(s, DEM_ERR_INVALID_ARG, "cell_scale must be finite and >= 1");
  if (t->member_scan != 0 && t->member_scan != 1)
    return fail(s, DEM_ERR_INVALID_ARG, "member_scan must be 0 or 1");
  if (t->member_read < 0 || t->member_read > 2)
    return fail(s, DEM_ERR_INVALID_ARG, "member_read must be 0, 1 or 2");
  if (t->fused < 0 || t->fused > 2) return fail(s, DEM_ERR_INVALID_ARG, "fused must be 0, 1 or 2");
  if (t->gravity_form < 0 || t->gravity_form > 2)
    return fail(s, DEM_ERR_INVALID_ARG, "gravity_form must be 0, 1 or 2");
  s->tune = *t;
  return DEM_OK;
}

int32_t dem_gravity_tiles(int32_t precision, int32_t* tiles, int32_t n_max) {
  int t[8];
  const int n = gravity_tiles(precision == 1 ? 1 : 0, t);
  for (int k = 0; k < n && k < n_max; ++k) tiles[k] = t[k];
  return n;
}

dem_status dem_set_profiling(dem_sim* s, int32_t enabled) {
  if (!s) return fail(nullptr, DEM_ERR_INVALID_ARG, "sim is NULL");
  if (enabled < 0 || enabled > 2) return fail(s, DEM_ERR_INVALID_ARG, "profiling must be 0, 1 or 2");
  s->profiling = enabled;
  s->prof_ms.assign(kNumStages, 0.0);
  s->prof_steps = 0;
  return DEM_OK;
}

dem_status dem_get_profile(const dem_sim* s, double* kernel_ms, int32_t n_max, int64_t* n_steps) {
  if (!s) return fail(nullptr, DEM_ERR_INVALID_ARG, "sim is NULL");
  for (int k = 0; k < n_max && k < kNumStages; ++k)
    kernel_ms[k] = k < (int)s->prof_ms.size() ? s->prof_ms[k] : 0.0;
  if (n_steps) *n_steps = s->prof_steps;
  return DEM_OK;
}

const char* dem_profile_names(void) { return kStageNames; }

dem_status dem_sim_status(const dem_sim* s) {
  if (!s) return DEM_ERR_INVALID_ARG;
  return status_code(s->h.status);
}

// ---------------------------------------------------------------------------
// stateless contact search
// ---------------------------------------------------------------------------

dem_status dem_find_contacts(const double* pos, const double* radius, const int32_t* agg,
                             int64_t n, const double* box, uint64_t* pairs_out, int64_t cap,
                             int64_t* n_out) {
  if (!n_out || n < 0 || cap < 0 || (cap > 0 && !pairs_out))
    return fail(nullptr, DEM_ERR_INVALID_ARG, "bad argument");
  if (n == 0) {                 // no spheres, no contacts
    *n_out = 0;
    return DEM_OK;
  }
  if (!pos || !radius || !agg) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad argument");
  if (n > (int64_t(1) << 28)) return fail(nullptr, DEM_ERR_INVALID_ARG, "too many spheres");
  if (require_device(nullptr) != DEM_OK) return DEM_ERR_DEVICE;
  double smax = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!(radius[i] > 0) || !std::isfinite(radius[i])) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad radius");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(pos[3 * i + k])) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad position");
    smax = std::max(smax, radius[i]);
  }
  dem_params p{};
  p.dt = 1.0;
  p.k_n = p.k_t = 1.0;
  p.eps_n = p.eps_t = 1.0;
  p.periodic = box ? 1 : 0;
  if (box) {
    p.box[0] = p.box[1] = p.box[2] = box[0];
    if (!(box[0] > 0)) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad box");
  }
  p.max_contacts_per_sphere = kFindContactsCap;
  dem_sim* s = nullptr;
  dem_status r = dem_create(&p, nullptr, nullptr, &s);
  if (r != DEM_OK) return r;
  struct Guard {
    dem_sim* s;
    ~Guard() { dem_destroy(s); }
  } guard{s};
  // one sphere per pseudo-aggregate; the given ids decide which pairs count
  r = alloc_pile(s, n, n);
  if (r != DEM_OK) return fail(nullptr, r, s->err);
  PileDev& h = s->h;
  h.na = 0;   // positions are given: reconstruction only measures the bbox
  h.cell_min = 2.0 * smax;
  if (box) h.n_periodic = periodic_cells(box[0], h.cell_min, h.bits);
  hipStream_t st = nullptr;
  std::vector<double> col(3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) col[k * n + i] = pos[3 * i + k];
  std::vector<double> ones(n, 1.0);
  HIPCHK(s, hipMemcpyAsync(h.r, col.data(), 3 * n * 8, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(h.s, radius, n * 8, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(h.m, ones.data(), n * 8, hipMemcpyHostToDevice, st));
  HIPCHK(s, hipMemcpyAsync(h.agg, agg, n * 4, hipMemcpyHostToDevice, st));
  launch_fill_u32(st, h.cell_cnt, 0u, s->sz.cells + 1);
  r = ensure_own_table(s);
  if (r != DEM_OK) return fail(nullptr, r, s->err);
  HIPCHK(s, put_entry(s, s->own.d_table, st));
  r = rebuild(s->own, st, s);
  if (r != DEM_OK) return fail(nullptr, r, s->err);
  Batch& b = s->own;
  launch_reconstruct(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_grid(st, b.d_table, 1, kModeInit, 1.0);
  launch_bin(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_scan(st, b.seg_cells, b.n_seg_cells, b.item_cells, b.n_item_cells, b.sums_cells,
              b.max_items_cells);
  launch_scatter(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_cell_sort(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_search(st, b.d_table, b.wl_sph, b.n_sph_blk, 0);
  launch_scan(st, b.seg_pairs, b.n_seg_pairs, b.item_pairs, b.n_item_pairs, b.sums_pairs,
              b.max_items_pairs);
  launch_search(st, b.d_table, b.wl_sph, b.n_sph_blk, 1);
  HIPCHK(s, hipGetLastError());
  PileDev tmp;
  HIPCHK(s, hipMemcpyAsync(&tmp, b.d_table, sizeof(PileDev), hipMemcpyDeviceToHost, st));
  std::vector<uint32_t> off(n + 1);
  HIPCHK(s, hipMemcpyAsync(off.data(), h.up_off[1], (n + 1) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  const int64_t total = off[n];
  *n_out = total;
  if (tmp.status & kStCapacity) return fail(nullptr, DEM_ERR_CAPACITY, "more than 64 contacts per sphere");
  if (tmp.status != 0) return fail(nullptr, DEM_ERR_INVALID_ARG, "non-finite positions");
  std::vector<uint32_t> pj(std::max<int64_t>(total, 1));
  if (total) HIPCHK(s, hipMemcpy(pj.data(), h.pair_j[1], total * 4, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n; ++i)
    for (uint32_t q = off[i]; q < off[i + 1] && q < cap; ++q)
      pairs_out[q] = (uint64_t(i) << 32) | pj[q];
  return DEM_OK;
}

dem_status dem_find_contacts_noalloc(const double* pos, const double* radius,
                                     const int32_t* agg, int64_t n, const double* box,
                                     uint64_t* pairs_out, int64_t cap, int64_t* n_out,
                                     void* hip_stream) {
  if (!n_out || n < 0 || cap < 0 || (cap > 0 && !pairs_out))
    return fail(nullptr, DEM_ERR_INVALID_ARG, "bad argument");
  if (n > kNoAllocMaxSpheres)
    return fail(nullptr, DEM_ERR_INVALID_ARG,
                "more spheres than the static scratch holds (65536)");
  if (box && !(box[0] > 0 && std::isfinite(box[0])))
    return fail(nullptr, DEM_ERR_INVALID_ARG, "bad box");
  *n_out = 0;
  if (n == 0) return DEM_OK;
  if (!pos || !radius || !agg) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad argument");
  if (require_device(nullptr) != DEM_OK) return DEM_ERR_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  int dev = 0;
  HIPCHK(nullptr, hipGetDevice(&dev));
  void* base = nullptr;
  HIPCHK(nullptr, noalloc_scratch(dev, &base));
  PileDev h{};
  const NoAllocPlan q = plan_noalloc(static_cast<char*>(base), n, h);
  if (q.bytes > kNoAllocScratchBytes)
    return fail(nullptr, DEM_ERR_INVALID_ARG, "search does not fit the static scratch");
  // positions in, radius checks and the largest radius out
  launch_fill_u32(st, reinterpret_cast<uint32_t*>(q.hdr), 0u, sizeof(NoAllocHdr) / 4);
  hipLaunchKernelGGL(k_noalloc_ingest, dim3(q.n_blk), dim3(kBlock), 0, st, pos, radius, (int)n,
                     h.r, q.hdr);
  NoAllocHdr hdr{};
  HIPCHK(nullptr, hipMemcpyAsync(&hdr, q.hdr, sizeof hdr, hipMemcpyDeviceToHost, st));
  HIPCHK(nullptr, hipStreamSynchronize(st));
  if (hdr.bad) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad radius or position");
  double smax;
  std::memcpy(&smax, &hdr.max_r_bits, sizeof smax);
  // the table entry of a pile of given positions (no aggregates, no gravity)
  h.na = 0;
  h.ns = (int32_t)n;
  h.cap_pairs = (int32_t)kNoAllocMaxPairs;
  h.bits = choose_bits(n);
  h.periodic = box ? 1 : 0;
  h.box = box ? box[0] : 0.0;
  h.n_rblk = q.n_blk;
  h.cell_min = 2.0 * smax;
  h.s_cut = INFINITY;
  h.s_small = smax;
  h.n_big = 0;
  h.fail_step = -1;
  h.s = const_cast<double*>(radius);
  h.agg = const_cast<int32_t*>(agg);
  if (box) h.n_periodic = periodic_cells(box[0], h.cell_min, h.bits);
  // work lists and scan segments (fixed-size host staging)
  WorkItem wl[kNoAllocMaxSpheres / kBlock];
  for (int b = 0; b < q.n_blk; ++b) wl[b] = WorkItem{0, b * kBlock};
  ScanSeg sc{};
  sc.in = h.cell_cnt;
  sc.out_pp[0] = sc.out_pp[1] = h.cell_start;
  sc.n = (int32_t)(q.cells + 1);
  sc.n_items = q.n_item_cells;
  ScanItem ic[(((int64_t(1) << 18) + 1) + kScanChunk - 1) / kScanChunk];
  static_assert(sizeof(ic) / sizeof(ic[0]) >= (size_t)(((int64_t(1) << 18) + 1 + kScanChunk - 1) /
                                                        kScanChunk), "cell scan items");
  for (int c = 0; c < q.n_item_cells; ++c) ic[c] = ScanItem{0, c};
  ScanSeg sp[2]{};
  ScanItem ip[2 * ((kNoAllocMaxSpheres + kScanChunk - 1) / kScanChunk)];
  const uint32_t* ins[2] = {h.cnt_up, h.cnt_lo};
  uint32_t* outs[2] = {h.up_off[1], h.lo_off};
  for (int g = 0; g < 2; ++g) {
    sp[g].in = ins[g];
    sp[g].out_pp[0] = sp[g].out_pp[1] = outs[g];
    sp[g].n = (int32_t)n;
    sp[g].item0 = g * q.max_items_pairs;
    sp[g].n_items = q.max_items_pairs;
    for (int c = 0; c < q.max_items_pairs; ++c) ip[g * q.max_items_pairs + c] = ScanItem{g, c};
  }
  HIPCHK(nullptr, hipMemcpyAsync(q.entry, &h, sizeof h, hipMemcpyHostToDevice, st));
  HIPCHK(nullptr, hipMemcpyAsync(q.wl, wl, q.n_blk * sizeof(WorkItem), hipMemcpyHostToDevice, st));
  HIPCHK(nullptr, hipMemcpyAsync(q.seg_cells, &sc, sizeof sc, hipMemcpyHostToDevice, st));
  HIPCHK(nullptr, hipMemcpyAsync(q.item_cells, ic, q.n_item_cells * sizeof(ScanItem),
                                 hipMemcpyHostToDevice, st));
  HIPCHK(nullptr, hipMemcpyAsync(q.seg_pairs, sp, sizeof sp, hipMemcpyHostToDevice, st));
  HIPCHK(nullptr, hipMemcpyAsync(q.item_pairs, ip, q.n_item_pairs * sizeof(ScanItem),
                                 hipMemcpyHostToDevice, st));
  // the cell counts start at zero (the scatter returns them to zero)
  launch_fill_u32(st, h.cell_cnt, 0u, q.cells + 1);
  const PileDev* t = q.entry;
  launch_reconstruct(st, t, q.wl, q.n_blk);
  launch_grid(st, t, 1, kModeInit, 1.0);
  launch_bin(st, t, q.wl, q.n_blk);
  launch_scan(st, q.seg_cells, 1, q.item_cells, q.n_item_cells, q.sums_cells, q.max_items_cells);
  launch_scatter(st, t, q.wl, q.n_blk);
  launch_cell_sort(st, t, q.wl, q.n_blk);
  launch_search(st, t, q.wl, q.n_blk, 0);
  launch_scan(st, q.seg_pairs, 2, q.item_pairs, q.n_item_pairs, q.sums_pairs, q.max_items_pairs);
  launch_search(st, t, q.wl, q.n_blk, 1);
  HIPCHK(nullptr, hipGetLastError());
  int32_t status = 0;
  uint32_t total = 0;
  HIPCHK(nullptr, hipMemcpyAsync(&status, &q.entry->status, sizeof status, hipMemcpyDeviceToHost, st));
  HIPCHK(nullptr, hipMemcpyAsync(&total, h.up_off[1] + n, sizeof total, hipMemcpyDeviceToHost, st));
  HIPCHK(nullptr, hipStreamSynchronize(st));
  *n_out = total;
  if (status & kStCapacity)
    return fail(nullptr, DEM_ERR_CAPACITY, "more contacts than the static scratch holds");
  if (status != 0) return fail(nullptr, DEM_ERR_INVALID_ARG, "non-finite positions");
  if (cap > 0 && total > 0) {
    hipLaunchKernelGGL(k_noalloc_keys, dim3(q.n_blk), dim3(kBlock), 0, st, h.up_off[1], h.pair_j[1],
                       (int)n, pairs_out, cap);
    HIPCHK(nullptr, hipGetLastError());
    HIPCHK(nullptr, hipStreamSynchronize(st));
  }
  return DEM_OK;
}

// ---------------------------------------------------------------------------
// contact forces of given sphere states (same-input test hook)
// ---------------------------------------------------------------------------

dem_status dem_contact_forces(const dem_params* params, int64_t n, const double* pos,
                              const double* vel, const double* radius, const int32_t* agg,
                              int64_t n_agg, const double* agg_mass, const double* agg_spin,
                              int64_t n_old, const uint64_t* old_keys, const double* old_hist,
                              double* force, double* torque, uint64_t* keys_out,
                              double* hist_out, int64_t cap, int64_t* n_out) {
  std::string why;
  if (valid_params(params, &why) != DEM_OK) return fail(nullptr, DEM_ERR_INVALID_ARG, why);
  if (!n_out || n <= 0 || n_agg <= 0 || cap < 0 || n_old < 0 || !pos || !vel || !radius ||
      !agg || !agg_mass || !agg_spin || !force || !torque || (cap > 0 && (!keys_out || !hist_out)) ||
      (n_old > 0 && (!old_keys || !old_hist)))
    return fail(nullptr, DEM_ERR_INVALID_ARG, "bad argument");
  if (n > (int64_t(1) << 28) || n_agg > n) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad size");
  for (int64_t i = 0; i < n; ++i) {
    if (!(radius[i] > 0) || !std::isfinite(radius[i]) || agg[i] < 0 || agg[i] >= n_agg)
      return fail(nullptr, DEM_ERR_INVALID_ARG, "bad radius or aggregate id");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(pos[3 * i + k]) || !std::isfinite(vel[3 * i + k]))
        return fail(nullptr, DEM_ERR_INVALID_ARG, "non-finite position or velocity");
  }
  for (int64_t a = 0; a < n_agg; ++a) {
    if (!(agg_mass[a] > 0) || !std::isfinite(agg_mass[a]))
      return fail(nullptr, DEM_ERR_INVALID_ARG, "aggregate mass must be finite and > 0");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(agg_spin[3 * a + k])) return fail(nullptr, DEM_ERR_INVALID_ARG, "bad spin");
  }
  for (int64_t p = 0; p < n_old; ++p) {
    const uint64_t key = old_keys[p];
    const int64_t i = int64_t(key >> 32), j = int64_t(key & 0xffffffffu);
    if (i >= n || j <= i || j >= n + params->n_walls || (p > 0 && key <= old_keys[p - 1]))
      return fail(nullptr, DEM_ERR_INVALID_ARG, "old keys must be canonical and sorted");
  }
  if (require_device(nullptr) != DEM_OK) return DEM_ERR_DEVICE;
  dem_params p = *params;
  p.G = 0.0;                       // contacts only
  if (p.max_contacts_per_sphere <= 0) p.max_contacts_per_sphere = 16;
  dem_sim* s = nullptr;
  dem_status r = dem_create(&p, nullptr, nullptr, &s);
  if (r != DEM_OK) return r;
  struct Guard {
    dem_sim* s;
    ~Guard() { dem_destroy(s); }
  } guard{s};
  if (n_old > int64_t(s->c_max) * n) return fail(nullptr, DEM_ERR_CAPACITY, "too many old contacts");
  double s_cut, s_small;
  int n_big;
  split_big(radius, n, &s_cut, &s_small, &n_big);
  r = alloc_pile(s, n_agg, n);
  if (r != DEM_OK) return fail(nullptr, r, s->err);
  PileDev& h = s->h;
  h.given = 1;
  h.cell_min = 2.0 * s_small;
  h.s_cut = s_cut;
  h.s_small = s_small;
  h.n_big = n_big;
  if (p.periodic) h.n_periodic = periodic_cells(p.box[0], h.cell_min, h.bits);
  hipStream_t st = nullptr;
  auto put_cols = [&](double* d, const double* host, int k, int64_t m) -> hipError_t {
    std::vector<double> col(size_t(k) * m);
    for (int64_t i = 0; i < m; ++i)
      for (int c = 0; c < k; ++c) col[size_t(c) * m + i] = host[i * k + c];
    hipError_t e = hipMemcpyAsync(d, col.data(), col.size() * 8, hipMemcpyHostToDevice, st);
    return e == hipSuccess ? hipStreamSynchronize(st) : e;
  };
  HIPCHK(s, put_cols(h.r, pos, 3, n));
  HIPCHK(s, put_cols(h.v, vel, 3, n));
  HIPCHK(s, put_cols(h.wA, agg_spin, 3, n_agg));
  HIPCHK(s, hipMemcpy(h.s, radius, n * 8, hipMemcpyHostToDevice));
  HIPCHK(s, hipMemcpy(h.agg, agg, n * 4, hipMemcpyHostToDevice));
  HIPCHK(s, hipMemcpy(h.M, agg_mass, n_agg * 8, hipMemcpyHostToDevice));
  // the previous contact list (parity 0) with its spring history
  std::vector<uint32_t> off(n + 1, 0), pj(std::max<int64_t>(n_old, 1));
  for (int64_t q = 0; q < n_old; ++q) {
    off[(old_keys[q] >> 32) + 1]++;
    pj[q] = uint32_t(old_keys[q] & 0xffffffffu);
  }
  for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
  HIPCHK(s, hipMemcpy(h.up_off[0], off.data(), (n + 1) * 4, hipMemcpyHostToDevice));
  if (n_old) {
    HIPCHK(s, hipMemcpy(h.pair_j[0], pj.data(), n_old * 4, hipMemcpyHostToDevice));
    std::vector<double> col(n_old);
    for (int c = 0; c < kHist; ++c) {
      for (int64_t q = 0; q < n_old; ++q) col[q] = old_hist[q * kHist + c];
      HIPCHK(s, hipMemcpy(h.hist[0] + size_t(c) * h.cap_pairs, col.data(), n_old * 8,
                          hipMemcpyHostToDevice));
    }
  }
  launch_fill_u32(st, h.cell_cnt, 0u, s->sz.cells + 1);
  r = ensure_own_table(s);
  if (r != DEM_OK) return fail(nullptr, r, s->err);
  HIPCHK(s, put_entry(s, s->own.d_table, st));
  r = rebuild(s->own, st, s);
  if (r != DEM_OK) return fail(nullptr, r, s->err);
  // one evaluation pass without motion, gravity or the aggregate reduction
  Batch& b = s->own;
  launch_reconstruct(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_grid(st, b.d_table, 1, kModeInit, p.dt);
  launch_bin(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_scan(st, b.seg_cells, b.n_seg_cells, b.item_cells, b.n_item_cells, b.sums_cells,
              b.max_items_cells);
  launch_scatter(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_cell_sort(st, b.d_table, b.wl_sph, b.n_sph_blk);
  launch_search(st, b.d_table, b.wl_sph, b.n_sph_blk, 0);
  if (b.n_big_blk) launch_search_big(st, b.d_table, b.wl_big, b.n_big_blk, 0);
  launch_scan(st, b.seg_pairs, b.n_seg_pairs, b.item_pairs, b.n_item_pairs, b.sums_pairs,
              b.max_items_pairs);
  launch_search(st, b.d_table, b.wl_sph, b.n_sph_blk, 1);
  if (b.n_big_blk) launch_search_big(st, b.d_table, b.wl_big, b.n_big_blk, 1);
  launch_forces(st, b.d_table, b.wl_sph, b.n_sph_blk, b.cp, b.precision);
  HIPCHK(s, hipGetLastError());
  PileDev tmp;
  HIPCHK(s, hipMemcpyAsync(&tmp, b.d_table, sizeof(PileDev), hipMemcpyDeviceToHost, st));
  std::vector<uint32_t> off1(n + 1);
  HIPCHK(s, hipMemcpyAsync(off1.data(), h.up_off[1], (n + 1) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(s, hipStreamSynchronize(st));
  const int64_t total = off1[n];
  *n_out = total;
  if (tmp.status & kStCapacity) return fail(nullptr, DEM_ERR_CAPACITY, "contact capacity exceeded");
  if (tmp.status != 0) return fail(nullptr, DEM_ERR_UNSTABLE, "non-finite force or bad positions");
  r = fetch_rows(s, h.F, 3, n, force, st);
  if (r == DEM_OK) r = fetch_rows(s, h.tau, 3, n, torque, st);
  if (r != DEM_OK) return fail(nullptr, r, s->err);
  if (cap > 0 && total > 0) {
    std::vector<uint32_t> pj1(total);
    HIPCHK(s, hipMemcpy(pj1.data(), h.pair_j[1], total * 4, hipMemcpyDeviceToHost));
    std::vector<double> hh(size_t(kHist) * h.cap_pairs);
    HIPCHK(s, hipMemcpy(hh.data(), h.hist[1], hh.size() * 8, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i)
      for (uint32_t q = off1[i]; q < off1[i + 1] && q < cap; ++q) {
        keys_out[q] = (uint64_t(i) << 32) | pj1[q];
        for (int c = 0; c < kHist; ++c) hist_out[q * kHist + c] = hh[size_t(c) * h.cap_pairs + q];
      }
  }
  return DEM_OK;
}

// ---------------------------------------------------------------------------
// engine
// ---------------------------------------------------------------------------

dem_status dem_engine_create(size_t budget, void* hip_stream, dem_engine** out) {
  if (!out) return fail(nullptr, DEM_ERR_INVALID_ARG, "out is NULL");
  dem_engine* e = new dem_engine();
  e->budget = budget;
  e->stream = static_cast<hipStream_t>(hip_stream);
  *out = e;
  return DEM_OK;
}

namespace {

bool same_contact_model(const dem_params& a, const dem_params& b) {
  return a.dt == b.dt && a.k_n == b.k_n && a.k_t == b.k_t && a.eps_n == b.eps_n &&
         a.eps_t == b.eps_t && a.mu_s == b.mu_s && a.mu_r == b.mu_r && a.mu_t == b.mu_t &&
         a.k_r == b.k_r && a.k_q == b.k_q && a.precision == b.precision &&
         a.max_overlap_frac == b.max_overlap_frac;
}

dem_status engine_table(dem_engine* e, dem_sim* errsim) {
  Batch& b = e->batch;
  const int n = (int)b.members.size();
  if (n > b.table_cap) {
    int nc = std::max(16, b.table_cap * 2);
    while (nc < n) nc *= 2;
    PileDev* t = nullptr;
    HIPCHK(errsim, hipMalloc(&t, size_t(nc) * sizeof(PileDev)));
    if (b.d_table) {
      HIPCHK(errsim, hipMemcpyAsync(t, b.d_table, size_t(b.table_cap) * sizeof(PileDev),
                                    hipMemcpyDeviceToDevice, e->stream));
      HIPCHK(errsim, hipStreamSynchronize(e->stream));
      (void)hipFree(b.d_table);
    }
    b.d_table = t;
    b.table_cap = nc;
  }
  return DEM_OK;
}

}  // namespace

dem_status dem_engine_attach(dem_engine* e, dem_sim* s) {
  if (!e || !s) return fail(s, DEM_ERR_INVALID_ARG, "NULL argument");
  if (s->engine) return fail(s, DEM_ERR_STATE, "already attached");
  if (!s->has_aggs) return fail(s, DEM_ERR_STATE, "no aggregates");
  if (s->h.status != 0) return fail(s, DEM_ERR_STATE, "system has failed; restore it first");
  if (!e->batch.members.empty() && !same_contact_model(e->batch.members[0]->prm, s->prm))
    return fail(s, DEM_ERR_INVALID_ARG, "contact model or time step differs from the engine's");
  if (e->used + s->bytes > e->budget) return fail(s, DEM_ERR_OOM, "engine memory budget exceeded");
  // settle the system's own work, then move its table entry into the engine
  HIPCHK(s, get_entry(s, s->own.d_table, s->stream));
  Batch& b = e->batch;
  b.members.push_back(s);
  dem_status r = engine_table(e, s);
  if (r != DEM_OK) {
    b.members.pop_back();
    return r;
  }
  const int slot = (int)b.members.size() - 1;
  HIPCHK(s, put_entry(s, b.d_table + slot, e->stream));
  s->engine = e;
  s->engine_slot = slot;
  e->used += s->bytes;
  b.cp = contact_params(b.members[0]->prm);
  b.precision = b.members[0]->prm.precision;
  b.dirty = true;
  return DEM_OK;
}

dem_status dem_engine_detach(dem_engine* e, dem_sim* s) {
  if (!e || !s) return fail(s, DEM_ERR_INVALID_ARG, "NULL argument");
  if (s->engine != e) return fail(s, DEM_ERR_STATE, "not attached to this engine");
  Batch& b = e->batch;
  HIPCHK(s, hipStreamSynchronize(e->stream));
  HIPCHK(s, get_entry(s, b.d_table + s->engine_slot, e->stream));
  // compact the table: move later entries down by one
  const int slot = s->engine_slot;
  for (int k = slot + 1; k < (int)b.members.size(); ++k) {
    dem_sim* o = b.members[k];
    HIPCHK(s, get_entry(o, b.d_table + k, e->stream));
    HIPCHK(s, put_entry(o, b.d_table + k - 1, e->stream));
    o->engine_slot = k - 1;
  }
  b.members.erase(b.members.begin() + slot);
  e->used -= s->bytes;
  s->engine = nullptr;
  s->engine_slot = -1;
  HIPCHK(s, put_entry(s, s->own.d_table, s->stream));
  HIPCHK(s, hipStreamSynchronize(e->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  b.dirty = true;
  return DEM_OK;
}

dem_status dem_engine_step(dem_engine* e, int64_t n_steps) {
  if (!e) return fail(nullptr, DEM_ERR_INVALID_ARG, "engine is NULL");
  Batch& b = e->batch;
  if (b.members.empty() || n_steps <= 0) return DEM_OK;
  if (b.dirty) {
    dem_status r = rebuild(b, e->stream, b.members[0]);
    if (r != DEM_OK) return r;
  }
  if (e->profiling) {
    dem_status r = profiled_passes(b, e->stream, n_steps, e->events, e->prof_ms, e->prof_steps,
                                   b.members[0]);
    if (r != DEM_OK) return r;
  } else {
    dem_status r = ensure_graph(b, e->stream, b.members[0]);
    if (r != DEM_OK) return r;
    for (int64_t k = 0; k < n_steps; ++k) {
      hipError_t he = hipGraphLaunch(b.graph, e->stream);
      if (he != hipSuccess)
        return fail(b.members[0], DEM_ERR_DEVICE, hip_msg(he, "hipGraphLaunch"));
    }
  }
  // one read-back of every entry's bookkeeping
  std::vector<PileDev> tab(b.members.size());
  hipError_t he = hipMemcpyAsync(tab.data(), b.d_table, tab.size() * sizeof(PileDev),
                                 hipMemcpyDeviceToHost, e->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
  if (he != hipSuccess) return fail(b.members[0], DEM_ERR_DEVICE, hip_msg(he, "engine read-back"));
  dem_status first = DEM_OK;
  for (size_t k = 0; k < b.members.size(); ++k) {
    dem_sim* s = b.members[k];
    copy_device_fields(s->h, tab[k]);
    s->stepped = true;
    const dem_status c = status_code(s->h.status);
    if (c < 0 && first == DEM_OK) first = c;     // a stopped system is not a failure
  }
  return first;
}

dem_status dem_engine_set_profiling(dem_engine* e, int32_t enabled) {
  if (!e) return fail(nullptr, DEM_ERR_INVALID_ARG, "engine is NULL");
  e->profiling = enabled != 0;
  e->prof_ms.assign(kNumStages, 0.0);
  e->prof_steps = 0;
  return DEM_OK;
}

dem_status dem_engine_get_profile(const dem_engine* e, double* kernel_ms, int32_t n_max,
                                  int64_t* n_steps) {
  if (!e) return fail(nullptr, DEM_ERR_INVALID_ARG, "engine is NULL");
  for (int k = 0; k < n_max && k < kNumStages; ++k)
    kernel_ms[k] = k < (int)e->prof_ms.size() ? e->prof_ms[k] : 0.0;
  if (n_steps) *n_steps = e->prof_steps;
  return DEM_OK;
}

dem_status dem_engine_destroy(dem_engine* e) {
  if (!e) return DEM_OK;
  for (hipEvent_t ev : e->events) (void)hipEventDestroy(ev);
  while (!e->batch.members.empty()) dem_engine_detach(e, e->batch.members.back());
  free_meta(e->batch);
  release_side(e->batch);
  if (e->batch.d_table) (void)hipFree(e->batch.d_table);
  delete e;
  return DEM_OK;
}

}  // extern "C"
