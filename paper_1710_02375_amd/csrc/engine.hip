// Host engine behind the C ABI of include/lbm.h: instance tables, device
// memory layout, work lists, the per-step launch schedule (optionally replayed
// from a captured hipGraph), synchronous queries and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"

using namespace kbc;

// Workgroups of the FP64 pass over deferred near-equilibrium nodes.
static constexpr int kFixupBlocks = 512;
// Upper bound on the one-wavefront workgroups of a boundary launch.
static constexpr int kBoundaryWorkgroups = 4096;

// Static workspace of lbm_wall_force_noalloc: quadrature points, normals,
// weights and tractions (3 D + 1 doubles per point, D <= 3), the force
// kernel's partial sums (four doubles per workgroup of at least four points)
// and the reduced sums, for up to kNoAllocMaxPoints points.  5.8 MB, held by
// every GPU the library runs on until the process ends.
static constexpr int kNoAllocMaxPoints = 65536;
static constexpr size_t kForceScratchDoubles =
    (size_t)kNoAllocMaxPoints * 10 + ((size_t)kNoAllocMaxPoints / 4 + 1) * 4 + 8;
static __device__ __align__(256) double scratch[kForceScratchDoubles];

struct lbm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // Boundary kernels beside the bulk kernel: the scan, wavefront and wall
  // kernels on `side`, forked from and joined back to `stream` every step
  // (KBC_SERIAL_BOUNDARY=1 keeps everything on `stream`).  One side stream:
  // a captured graph then has two branches, which run on two queues.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = true;
  void* (*ualloc)(size_t, void*) = nullptr;
  void (*ufree)(void*, void*) = nullptr;
  void* actx = nullptr;
  int use_graph = 1;

  int Q = 27, D = 3, storage = LBM_F32, esize = 4;
  const Ops* ops = nullptr;
  int n_inst = 0;
  std::vector<lbm_instance_desc> desc;
  std::vector<InstDev> hinst;
  std::vector<int> moving;        // body moves (geometry changes every step)
  std::vector<char> has_body;
  std::vector<char> has_faces;    // an inflow or outflow face
  bool any_faces = false;
  std::vector<char> force_valid;
  // Device arrays of surface-mesh bodies, per instance (grown on demand).
  struct MeshBuf {
    double* v = nullptr;   size_t v_cap = 0;    // positions then velocities
    int* f = nullptr;      size_t f_cap = 0;    // faces
    int* cs = nullptr;     size_t cs_cap = 0;   // column starts
    double* cx = nullptr;  size_t cx_cap = 0;   // column crossings
    int* bs = nullptr;     size_t bs_cap = 0;   // cell starts
    int* bf = nullptr;     size_t bf_cap = 0;   // cell faces
  };
  std::vector<MeshBuf> mesh;
  // Multiphase (Sec. III.B): the fields of every instance (density, phi,
  // Laplacian; 3 N elements each, FP64 for FP64 storage, else FP32), and
  // whether some instance has the forcing on (then every instance steps
  // through the multiphase pipeline, those with it off at zero force).
  void* mp_field = nullptr;
  bool any_mp = false;
  double* force_ws = nullptr;     // wall-force workspace, grown on demand
  size_t force_ws_doubles = 0;
  double* scratch = nullptr;      // device address of `scratch` on this device
  int64_t total_nodes = 0;
  size_t pop_elems = 0;           // elements per population buffer

  void* buf[2] = {nullptr, nullptr};
  int cur = 0;                    // buf[cur] holds the current state
  uint8_t* flags = nullptr;
  size_t flag_bytes = 0;
  InstDev* dinst = nullptr;
  int64_t* dclock = nullptr;
  uint32_t* derr = nullptr;
  uint32_t* herr = nullptr;       // pinned mirror of the error word
  // Near-equilibrium mask words (one per 64 nodes of a tile, the current
  // tiling's layout), set by the bulk kernel, read and cleared by the FP64
  // pass.
  uint64_t* dneq_words = nullptr;
  size_t neq_words_cap = 0;
  // Boundary node lists (two per launch: nodes with a cut link to a body,
  // then nodes whose missing populations all come from wall faces; inflow
  // and outflow plane nodes are formed by the bulk kernel): instance k's
  // pair starts at
  // 2 bl_off[k] (capacity bl_cap[k] each, its box-tile volume); the batched
  // launch uses the whole allocation with capacity bl_total.  Counter pairs:
  // [2k, 2k+1] per instance, [2 n_inst, 2 n_inst + 1] batched.
  uint2* dblist = nullptr;
  size_t dblist_cap = 0;
  uint32_t* dbcount = nullptr;
  std::vector<uint32_t> bl_off, bl_cap;
  uint32_t bl_total = 0;
  // Workgroups of the batched boundary launch: Grad wavefronts, wall-node
  // threads (64 per workgroup).
  int bl_nwg_all = 0, bl_nwall_all = 0;
  std::vector<int> bl_nwg, bl_nwall, bl_stat;   // per instance, and stats offsets
  int bstat_slots = 0;                // stats slots reserved for boundary launches
  hipEvent_t err_event = nullptr;
  bool err_pending = false;
  int64_t step = 0;

  int variant = 0;
  std::vector<Tile> tiles;
  std::vector<int> tile_first, tile_count;
  Tile* dtiles = nullptr;
  std::vector<Region> regions;
  std::vector<BoxTile> btiles, gtiles;
  std::vector<int> bt_first, bt_count;
  Region* dregions = nullptr;
  BoxTile* dbtiles = nullptr;
  BoxTile* dgtiles = nullptr;
  bool time_dependent = false;

  int stats_enabled = 0;
  StatPartial* dstats = nullptr;
  size_t dstats_cap = 0;
  int launch_mode = 0;

  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool graph_failed = false;
  std::string err;
};

namespace {

thread_local std::string g_create_error;

lbm_status fail(lbm_ctx* c, lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf; else g_create_error = buf;
  return s;
}

#define HIPCHECK(ctx, expr)                                                                    \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail((ctx), LBM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));       \
  } while (0)

// Device address of the static wall-force workspace on the context's device,
// resolved once per device (with that device current) and kept.  In host
// code `scratch` names a host-side stand-in, never the device memory.
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;

lbm_status resolve_scratch(lbm_ctx* c) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(c->device);
  if (it != g_scratch_ptr.end()) {
    c->scratch = it->second;
    return LBM_OK;
  }
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return fail(c, LBM_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
  }
  g_scratch_ptr[c->device] = static_cast<double*>(ptr);
  c->scratch = static_cast<double*>(ptr);
  return LBM_OK;
}

lbm_status dev_alloc(lbm_ctx* c, size_t bytes, void** p) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (c->ualloc) {
    *p = c->ualloc(bytes, c->actx);
    if (!*p) return fail(c, LBM_ERR_OOM, "allocator callback returned NULL for %zu bytes", bytes);
    return LBM_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(c, LBM_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return LBM_OK;
}

void dev_free(lbm_ctx* c, void* p) {
  if (!p) return;
  if (c->ufree) c->ufree(p, c->actx);
  else (void)hipFree(p);
}

template <typename T>
lbm_status upload(lbm_ctx* c, T** dptr, const std::vector<T>& h) {
  dev_free(c, *dptr);
  *dptr = nullptr;
  lbm_status st = dev_alloc(c, std::max<size_t>(h.size(), 1) * sizeof(T), (void**)dptr);
  if (st) return st;
  if (!h.empty())
    HIPCHECK(c, hipMemcpyAsync(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice,
                               c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int storage_bytes(int st) {
  switch (st) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    default: return 2;
  }
}

bool valid_faces(const lbm_instance_desc& d) {
  for (int k = 0; k < 6; ++k)
    if (d.face[k] < LBM_FACE_PERIODIC || d.face[k] > LBM_FACE_WALL) return false;
  for (int a = 0; a < 3; ++a) {
    const bool p0 = d.face[2 * a] == LBM_FACE_PERIODIC, p1 = d.face[2 * a + 1] == LBM_FACE_PERIODIC;
    if (p0 != p1) return false;
  }
  for (int k = 0; k < 6; ++k) {
    if (d.face[k] == LBM_FACE_INLET && k != 0) return false;
    if (d.face[k] == LBM_FACE_OUTLET && k != 1) return false;
  }
  if (d.lattice == LBM_D2Q9 && (d.face[4] != LBM_FACE_PERIODIC || d.face[5] != LBM_FACE_PERIODIC))
    return false;
  return true;
}

bool needs_flags(const lbm_instance_desc& d) {
  for (int k = 0; k < 6; ++k)
    if (d.face[k] != LBM_FACE_PERIODIC) return true;
  return false;
}

// Swept box of a body over its whole motion, with a 2-node margin; false if
// it leaves the domain along a periodic axis.
bool body_box(const lbm_ctx* c, int k, const lbm_body& b, int lo[3], int hi[3]) {
  const lbm_instance_desc& d = c->desc[k];
  const int n[3] = {d.nx, d.ny, d.nz};
  double blo[3] = {0, 0, 0}, bhi[3] = {(double)d.nx, (double)d.ny, (double)d.nz};
  const double* p = b.params;
  if (b.kind == LBM_BODY_SPHERE) {
    for (int a = 0; a < c->D; ++a) {
      blo[a] = p[a] - std::fabs(p[4 + a]) - p[3];
      bhi[a] = p[a] + std::fabs(p[4 + a]) + p[3];
    }
  } else if (b.kind == LBM_BODY_FLAP) {
    blo[0] = p[0] - 0.5 * p[2] - std::fabs(p[3]);
    bhi[0] = p[0] + 0.5 * p[2] + std::fabs(p[3]);
    blo[1] = p[6];
    bhi[1] = p[6] + p[1];
  } else if (b.kind == LBM_BODY_PLATES) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = 0;
      hi[a] = n[a];
    }
    return true;
  }
  for (int a = 0; a < 3; ++a) {
    if (a >= c->D) {
      lo[a] = 0;
      hi[a] = 1;
      continue;
    }
    int l = (int)std::floor(blo[a]) - 2, h = (int)std::ceil(bhi[a]) + 3;
    const bool periodic = d.face[2 * a] == LBM_FACE_PERIODIC;
    if (l < 0 || h > n[a]) {
      if (periodic) return false;
      l = std::max(l, 0);
      h = std::min(h, n[a]);
    }
    if (h <= l) {
      l = 0;
      h = 0;
    }
    lo[a] = l;
    hi[a] = h;
  }
  return true;
}

void invalidate_graphs(lbm_ctx* c) {
  for (int p = 0; p < 2; ++p)
    if (c->graph[p]) {
      (void)hipGraphExecDestroy(c->graph[p]);
      c->graph[p] = nullptr;
    }
}

void push_box_tiles(std::vector<BoxTile>& out, int region, const Region& r) {
  const int64_t vol = (int64_t)(r.hi[0] - r.lo[0]) * (r.hi[1] - r.lo[1]) * (r.hi[2] - r.lo[2]);
  for (int64_t s = 0; s < vol; s += 256) {
    BoxTile t;
    t.region = region;
    t.count = (int)std::min<int64_t>(256, vol - s);
    t.local0 = s;
    out.push_back(t);
  }
}

// Statistics slots: bulk tiles, boundary tiles, then the FP64-pass workgroups.
lbm_status ensure_stats(lbm_ctx* c) {
  const size_t need = c->tiles.size() + (size_t)c->bstat_slots + kFixupBlocks + 1;
  if (need <= c->dstats_cap) return LBM_OK;
  dev_free(c, c->dstats);
  c->dstats = nullptr;
  lbm_status st = dev_alloc(c, need * sizeof(StatPartial), (void**)&c->dstats);
  if (st) return st;
  c->dstats_cap = need;
  return LBM_OK;
}

// Rebuilds regions, boundary and geometry work lists, and the stats buffer.
lbm_status rebuild_work(lbm_ctx* c) {
  c->regions.clear();
  c->btiles.clear();
  c->gtiles.clear();
  c->bt_first.assign(c->n_inst, 0);
  c->bt_count.assign(c->n_inst, 0);
  c->time_dependent = false;
  std::vector<int> geom_region(c->n_inst, -1);
  for (int k = 0; k < c->n_inst; ++k) {
    const lbm_instance_desc& d = c->desc[k];
    const InstDev& I = c->hinst[k];
    const int first = (int)c->regions.size();
    const int n[3] = {d.nx, d.ny, d.nz};
    for (int f = 0; f < 6; ++f) {
      if (d.face[f] == LBM_FACE_PERIODIC) continue;
      Region r;
      r.inst = k;
      r.first = first;
      for (int a = 0; a < 3; ++a) {
        r.lo[a] = 0;
        r.hi[a] = n[a];
      }
      const int a = f / 2;
      if (f % 2 == 0) r.hi[a] = 1; else r.lo[a] = n[a] - 1;
      c->regions.push_back(r);
    }
    if (c->has_body[k]) {
      Region r;
      r.inst = k;
      r.first = first;
      for (int a = 0; a < 3; ++a) {
        r.lo[a] = I.box_lo[a];
        r.hi[a] = I.box_hi[a];
      }
      geom_region[k] = (int)c->regions.size();
      c->regions.push_back(r);
    }
    if (d.ramp_steps > 0 && d.face[0] == LBM_FACE_INLET) c->time_dependent = true;
    if (c->moving[k]) c->time_dependent = true;
  }
  for (int k = 0; k < c->n_inst; ++k) {
    c->bt_first[k] = (int)c->btiles.size();
    for (int r = 0; r < (int)c->regions.size(); ++r)
      if (c->regions[r].inst == k) push_box_tiles(c->btiles, r, c->regions[r]);
    c->bt_count[k] = (int)c->btiles.size() - c->bt_first[k];
    if (c->moving[k] && geom_region[k] >= 0)
      push_box_tiles(c->gtiles, geom_region[k], c->regions[geom_region[k]]);
  }
  // Boundary node lists and their launch shapes.
  {
    const int ng = boundary_nodes_per_workgroup(c->Q);
    auto nwg_for = [&](uint32_t cap) {
      return (int)std::min<uint64_t>(kBoundaryWorkgroups, (cap + ng - 1) / ng);
    };
    auto nwall_for = [&](uint32_t cap) {
      return (int)std::min<uint64_t>(kBoundaryWorkgroups, (cap + 63) / 64);
    };
    c->bl_off.assign(c->n_inst, 0);
    c->bl_cap.assign(c->n_inst, 0);
    c->bl_nwg.assign(c->n_inst, 0);
    c->bl_nwall.assign(c->n_inst, 0);
    c->bl_stat.assign(c->n_inst, 0);
    uint32_t off = 0;
    int sum_nwg = 0;
    // The Grad wavefront kernel serves nodes with a cut link to a body, the
    // wall kernel nodes with wall faces only: neither runs without them.
    bool any_body = false, any_wall = false;
    std::vector<char> has_wall(c->n_inst, 0);
    for (int k = 0; k < c->n_inst; ++k) {
      for (int f = 0; f < 6; ++f)
        if (c->desc[k].face[f] == LBM_FACE_WALL) has_wall[k] = 1;
      any_wall = any_wall || has_wall[k];
      any_body = any_body || c->has_body[k];
    }
    for (int k = 0; k < c->n_inst; ++k) {
      uint32_t cap = 0;
      for (int t = c->bt_first[k]; t < c->bt_first[k] + c->bt_count[k]; ++t) cap += c->btiles[t].count;
      c->bl_off[k] = off;
      c->bl_cap[k] = cap;
      c->bl_nwg[k] = c->has_body[k] ? nwg_for(cap) : 0;
      c->bl_nwall[k] = has_wall[k] ? nwall_for(cap) : 0;
      c->bl_stat[k] = sum_nwg;
      sum_nwg += c->bl_nwg[k] + c->bl_nwall[k];
      off += cap;
    }
    c->bl_total = off;
    c->bl_nwg_all = any_body ? nwg_for(off) : 0;
    c->bl_nwall_all = any_wall ? nwall_for(off) : 0;
    // Side stream of the boundary kernels (default priority, like `stream`),
    // made with the first boundary work: a periodic context has none.
    if ((any_body || any_wall) && !c->side &&
        hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess)
      return fail(c, LBM_ERR_DEVICE, "hipStreamCreate failed");
    c->bstat_slots = std::max(c->bl_nwg_all + c->bl_nwall_all, sum_nwg);
    if ((size_t)off > c->dblist_cap) {
      dev_free(c, c->dblist);
      c->dblist = nullptr;
      c->dblist_cap = 0;
      lbm_status st2 = dev_alloc(c, 2 * (size_t)off * sizeof(uint2), (void**)&c->dblist);
      if (st2) return st2;
      c->dblist_cap = off;
    }
  }
  lbm_status st;
  if ((st = upload(c, &c->dregions, c->regions))) return st;
  if ((st = upload(c, &c->dbtiles, c->btiles))) return st;
  if ((st = upload(c, &c->dgtiles, c->gtiles))) return st;
  if ((st = ensure_stats(c))) return st;
  invalidate_graphs(c);
  return LBM_OK;
}

lbm_status rebuild_tiles(lbm_ctx* c) {
  const int tsz = bulk_variant_tile(c->variant);
  c->tiles.clear();
  c->tile_first.assign(c->n_inst, 0);
  c->tile_count.assign(c->n_inst, 0);
  for (int k = 0; k < c->n_inst; ++k) {
    c->tile_first[k] = (int)c->tiles.size();
    const int64_t N = c->hinst[k].N;
    for (int64_t s = 0; s < N; s += tsz) {
      Tile t;
      t.inst = k;
      t.node0 = s;
      t.count = (int)std::min<int64_t>(tsz, N - s);
      c->tiles.push_back(t);
    }
    c->tile_count[k] = (int)c->tiles.size() - c->tile_first[k];
  }
  lbm_status st = upload(c, &c->dtiles, c->tiles);
  if (st) return st;
  // Mask words of the new tiling, cleared: the bulk kernel stores only words
  // with a deferred node and the FP64 pass clears them, so they stay zero
  // from here on (the FP64 pass also skips any bit beyond a tile's count).
  const size_t nw = c->tiles.size() * (size_t)(tsz / 64);
  if (nw > c->neq_words_cap) {
    dev_free(c, c->dneq_words);
    c->dneq_words = nullptr;
    c->neq_words_cap = 0;
    if ((st = dev_alloc(c, nw * sizeof(uint64_t), (void**)&c->dneq_words))) return st;
    c->neq_words_cap = nw;
  }
  HIPCHECK(c, hipMemsetAsync(c->dneq_words, 0, c->neq_words_cap * sizeof(uint64_t), c->stream));
  if ((st = ensure_stats(c))) return st;
  invalidate_graphs(c);
  return LBM_OK;
}

// Enqueues one step reading buf[src] and writing buf[1 - src].
lbm_status enqueue_step(lbm_ctx* c, int src) {
  StepBuffers b;
  b.insts = c->dinst;
  b.src = c->buf[src];
  b.dst = c->buf[1 - src];
  b.flags = c->flags;
  b.err = c->derr;
  b.clock = c->dclock;
  b.stats = c->stats_enabled ? c->dstats : nullptr;
  b.clock_tick = c->time_dependent ? c->dclock : nullptr;
  b.bcount = c->dbcount;
  b.nbcount = 2 * (c->n_inst + 1);
  // The multiphase pipeline defers nothing (FP64 collision throughout).
  b.neq_words = c->dneq_words;
  b.neq_wpt = (uint32_t)(bulk_variant_tile(c->variant) / 64);
  b.neq_nwords = c->any_mp ? 0u : (uint32_t)c->tiles.size() * b.neq_wpt;
  b.tiles = c->dtiles;
  const int ngt = (int)c->gtiles.size();
  if (ngt > 0)
    for (int stage = 0; stage < 3; ++stage)
      HIPCHECK(c, c->ops->geometry(stage, c->dinst, c->dregions, c->dgtiles, ngt, c->buf[src],
                                   c->flags, c->dclock, 1, c->stream));
  const int ntiles = (int)c->tiles.size();
  const int nbt = (int)c->btiles.size();
  // Multiphase: the boundary kernels write pre-collision states, then the
  // three multiphase passes stream, differentiate and collide.
  const bool mp = c->any_mp;
  if (c->launch_mode == 0) {
    // The boundary kernels and the bulk kernel read the same source buffer
    // and write disjoint nodes of the destination (the bulk kernel skips
    // every node the scan can list): without the multiphase passes, which
    // read what the boundary kernels write, they run side by side, the
    // latency-bound boundary work under the bandwidth-bound bulk.  Both
    // follow the geometry update (flags, refilled nodes); the FP64 pass
    // follows both.
    const bool fork = !mp && c->overlap && c->side && nbt > 0 &&
                      (c->bl_nwg_all > 0 || c->bl_nwall_all > 0);
    hipStream_t sb = c->stream;
    if (fork) {
      HIPCHECK(c, hipEventRecord(c->ev_fork, c->stream));
      HIPCHECK(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
      sb = c->side;
    }
    HIPCHECK(c, c->ops->boundary(b, c->dregions, c->dbtiles, 0, nbt, c->dblist, c->bl_total,
                                 c->dbcount + 2 * c->n_inst, c->bl_nwg_all, c->bl_nwall_all, ntiles,
                                 mp, sb));
    if (mp) {
      for (int stage = 0; stage < 3; ++stage)
        HIPCHECK(c, c->ops->mp(stage, b, c->dtiles, 0, ntiles, c->stream));
    } else {
      HIPCHECK(c, c->ops->bulk(c->variant, b, c->dtiles, 0, ntiles, c->any_faces, c->stream));
    }
    if (fork) {
      HIPCHECK(c, hipEventRecord(c->ev_join, c->side));
      HIPCHECK(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
    }
  } else {
    for (int k = 0; k < c->n_inst; ++k) {
      HIPCHECK(c, c->ops->boundary(b, c->dregions, c->dbtiles, c->bt_first[k], c->bt_count[k],
                                   c->dblist + 2 * (size_t)c->bl_off[k], c->bl_cap[k],
                                   c->dbcount + 2 * k, c->bl_nwg[k], c->bl_nwall[k],
                                   ntiles + c->bl_stat[k], mp, c->stream));
      if (!mp)
        HIPCHECK(c, c->ops->bulk(c->variant, b, c->dtiles, c->tile_first[k], c->tile_count[k],
                                 c->has_faces[k] != 0, c->stream));
    }
    // The multiphase passes read neighbouring fields, which the boundary
    // kernels of every instance write first.
    if (mp)
      for (int stage = 0; stage < 3; ++stage)
        for (int k = 0; k < c->n_inst; ++k)
          HIPCHECK(c, c->ops->mp(stage, b, c->dtiles, c->tile_first[k], c->tile_count[k],
                                 c->stream));
  }
  HIPCHECK(c, c->ops->fixup(b, kFixupBlocks, ntiles + c->bstat_slots, c->stream));
  return LBM_OK;
}

lbm_status ensure_graph(lbm_ctx* c, int parity) {
  if (c->graph[parity] || c->graph_failed) return LBM_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    c->graph_failed = true;
    return LBM_OK;
  }
  lbm_status s1 = enqueue_step(c, parity);
  lbm_status s2 = s1 ? s1 : enqueue_step(c, 1 - parity);
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (s2 || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    c->graph_failed = true;
    return s2;
  }
  e = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    c->graph[parity] = nullptr;
    c->graph_failed = true;
  }
  return LBM_OK;
}

lbm_status check_error_word(lbm_ctx* c) {
  uint32_t v = 0;
  HIPCHECK(c, hipMemcpyAsync(&v, c->derr, sizeof v, hipMemcpyDeviceToHost, c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  if (v) return fail(c, LBM_ERR_NONFINITE, "a node reached an invalid state (rho <= 0, |u| >= 1 or non-finite)");
  return LBM_OK;
}

lbm_status check_inst(lbm_ctx* c, int inst) {
  if (!c) return LBM_ERR_INVALID;
  if (inst < 0 || inst >= c->n_inst) return fail(c, LBM_ERR_INVALID, "instance %d out of range", inst);
  return LBM_OK;
}

// Runs the three geometry stages over the whole domain of instance k at the
// current time (set-up of a new body).
lbm_status full_geometry(lbm_ctx* c, int k) {
  std::vector<Region> reg(1);
  reg[0].inst = k;
  reg[0].first = 0;
  const lbm_instance_desc& d = c->desc[k];
  const int n[3] = {d.nx, d.ny, d.nz};
  for (int a = 0; a < 3; ++a) {
    reg[0].lo[a] = 0;
    reg[0].hi[a] = n[a];
  }
  std::vector<BoxTile> gt;
  push_box_tiles(gt, 0, reg[0]);
  Region* dr = nullptr;
  BoxTile* dg = nullptr;
  lbm_status st;
  if ((st = upload(c, &dr, reg))) return st;
  if ((st = upload(c, &dg, gt))) {
    dev_free(c, dr);
    return st;
  }
  for (int stage = 0; stage < 3 && !st; ++stage) {
    hipError_t e = c->ops->geometry(stage, c->dinst, dr, dg, (int)gt.size(), c->buf[c->cur],
                                    c->flags, c->dclock, 0, c->stream);
    if (e != hipSuccess) st = fail(c, LBM_ERR_DEVICE, "geometry kernel: %s", hipGetErrorString(e));
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  dev_free(c, dr);
  dev_free(c, dg);
  if (!st && e != hipSuccess) st = fail(c, LBM_ERR_DEVICE, "geometry sync: %s", hipGetErrorString(e));
  return st;
}

// ---------------------------------------------------------------------------
// Surface-mesh bodies: host-side indexes built at lbm_set_geometry (O(faces)
// work; the surface comes from the structure solver on the host).
// ---------------------------------------------------------------------------
struct MeshHost {
  std::vector<double> v;    // positions (3 per vertex) then velocities
  std::vector<int> f;       // faces (3 per face)
  std::vector<int> cs;      // column starts (ncols + 1)
  std::vector<double> cx;   // crossings, ascending per column
  std::vector<int> bs;      // cell starts (ncells + 1)
  std::vector<int> bf;      // faces per cell
  int col_lo[2], col_n[2];
  double bin_lo[3], bin_h;
  int bin_n[3];
};

// Crossings of the lattice lines along x (columns (y, z) of the box) with
// the surface.  3D: a column point inside a face's (y, z) projection, with a
// tie rule that gives a point on an edge shared by two faces to exactly one
// of them (edge functions evaluated in one canonical direction per edge);
// the crossing is the face's plane at that point.  2D: the even-odd rule with
// half-open y intervals per segment.
void mesh_columns(int D, const int box_lo[3], const int box_hi[3], MeshHost& m) {
  m.col_lo[0] = box_lo[1];
  m.col_n[0] = std::max(box_hi[1] - box_lo[1], 0);
  m.col_lo[1] = D == 3 ? box_lo[2] : 0;
  m.col_n[1] = D == 3 ? std::max(box_hi[2] - box_lo[2], 0) : 1;
  const size_t ncol = (size_t)m.col_n[0] * m.col_n[1];
  std::vector<std::vector<double>> col(ncol);
  const size_t nf = m.f.size() / 3;
  const double* V = m.v.data();
  auto push = [&](int y, int z, double x) {
    const int a = y - m.col_lo[0], b = z - m.col_lo[1];
    if (a < 0 || b < 0 || a >= m.col_n[0] || b >= m.col_n[1]) return;
    col[(size_t)a + (size_t)m.col_n[0] * b].push_back(x);
  };
  for (size_t k = 0; k < nf; ++k) {
    const int* fv = &m.f[3 * k];
    if (D == 2) {
      const double* p0 = V + 3 * fv[0];
      const double* p1 = V + 3 * fv[1];
      if (p0[1] == p1[1]) continue;
      const double ylo = std::min(p0[1], p1[1]), yhi = std::max(p0[1], p1[1]);
      for (int y = (int)std::ceil(ylo); (double)y < yhi; ++y)
        push(y, 0, p0[0] + ((double)y - p0[1]) * (p1[0] - p0[0]) / (p1[1] - p0[1]));
      continue;
    }
    // Projected vertices (u, w) = (y, z) and their x.
    double P[3][2], X[3];
    for (int j = 0; j < 3; ++j) {
      P[j][0] = V[3 * fv[j] + 1];
      P[j][1] = V[3 * fv[j] + 2];
      X[j] = V[3 * fv[j]];
    }
    auto edge = [&](const double* a, const double* b, double u, double w) {
      // cross(b - a, pt - a) evaluated from the lexicographically smaller end.
      const bool fwd = a[0] < b[0] || (a[0] == b[0] && a[1] < b[1]);
      const double* s0 = fwd ? a : b;
      const double* s1 = fwd ? b : a;
      const double e = (s1[0] - s0[0]) * (w - s0[1]) - (s1[1] - s0[1]) * (u - s0[0]);
      return fwd ? e : -e;
    };
    double area = edge(P[0], P[1], P[2][0], P[2][1]);
    if (area == 0.0) continue;
    int o[3] = {0, 1, 2};
    if (area < 0.0) std::swap(o[1], o[2]);   // counter-clockwise in (y, z)
    auto included = [&](const double* a, const double* b) {
      // Of an edge and its reverse exactly one is included.
      const double dw = b[1] - a[1], du = b[0] - a[0];
      return dw > 0.0 || (dw == 0.0 && du < 0.0);
    };
    const double umin = std::min({P[0][0], P[1][0], P[2][0]}), umax = std::max({P[0][0], P[1][0], P[2][0]});
    const double wmin = std::min({P[0][1], P[1][1], P[2][1]}), wmax = std::max({P[0][1], P[1][1], P[2][1]});
    for (int w = (int)std::ceil(wmin); (double)w <= wmax; ++w)
      for (int u = (int)std::ceil(umin); (double)u <= umax; ++u) {
        double E[3];
        bool in = true;
        for (int e = 0; e < 3 && in; ++e) {
          const double* a = P[o[e]];
          const double* b = P[o[(e + 1) % 3]];
          E[e] = edge(a, b, (double)u, (double)w);
          in = E[e] > 0.0 || (E[e] == 0.0 && included(a, b));
        }
        if (!in) continue;
        const double sum = E[0] + E[1] + E[2];
        if (!(sum > 0.0)) continue;
        // E[e] is the edge o[e] -> o[e+1]: weight of the opposite vertex.
        const double x = (E[1] * X[o[0]] + E[2] * X[o[1]] + E[0] * X[o[2]]) / sum;
        push(u, w, x);
      }
  }
  m.cs.assign(ncol + 1, 0);
  m.cx.clear();
  for (size_t k = 0; k < ncol; ++k) {
    std::sort(col[k].begin(), col[k].end());
    m.cs[k] = (int)m.cx.size();
    m.cx.insert(m.cx.end(), col[k].begin(), col[k].end());
  }
  m.cs[ncol] = (int)m.cx.size();
}

// Faces by cell of a uniform grid of spacing 2 over the surface's bounding
// box (one cell layer in z for 2D): each face listed in every cell its
// bounding box meets.
void mesh_cells(int D, MeshHost& m) {
  const size_t nv = m.v.size() / 6, nf = m.f.size() / 3;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (size_t i = 0; i < nv; ++i)
    for (int a = 0; a < D; ++a) {
      lo[a] = std::min(lo[a], m.v[3 * i + a]);
      hi[a] = std::max(hi[a], m.v[3 * i + a]);
    }
  m.bin_h = 2.0;
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      m.bin_lo[a] = -1.0;
      m.bin_n[a] = 1;
      continue;
    }
    m.bin_lo[a] = std::floor(lo[a]) - 2.0;
    m.bin_n[a] = std::max(1, (int)std::ceil((hi[a] + 2.0 - m.bin_lo[a]) / m.bin_h));
  }
  const size_t ncell = (size_t)m.bin_n[0] * m.bin_n[1] * m.bin_n[2];
  std::vector<std::vector<int>> cell(ncell);
  const int nc = D == 3 ? 3 : 2;
  for (size_t k = 0; k < nf; ++k) {
    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      double flo = 1e300, fhi = -1e300;
      for (int j = 0; j < nc; ++j) {
        flo = std::min(flo, m.v[3 * m.f[3 * k + j] + a]);
        fhi = std::max(fhi, m.v[3 * m.f[3 * k + j] + a]);
      }
      c0[a] = std::max(0, (int)std::floor((flo - m.bin_lo[a]) / m.bin_h));
      c1[a] = std::min(m.bin_n[a] - 1, (int)std::floor((fhi - m.bin_lo[a]) / m.bin_h));
    }
    for (int z = c0[2]; z <= c1[2]; ++z)
      for (int y = c0[1]; y <= c1[1]; ++y)
        for (int x = c0[0]; x <= c1[0]; ++x)
          cell[(size_t)x + (size_t)m.bin_n[0] * ((size_t)y + (size_t)m.bin_n[1] * z)].push_back((int)k);
  }
  m.bs.assign(ncell + 1, 0);
  m.bf.clear();
  for (size_t k = 0; k < ncell; ++k) {
    m.bs[k] = (int)m.bf.size();
    m.bf.insert(m.bf.end(), cell[k].begin(), cell[k].end());
  }
  m.bs[ncell] = (int)m.bf.size();
}

template <typename T>
lbm_status ensure_dev(lbm_ctx* c, T** p, size_t* cap, size_t need) {
  if (need <= *cap && *p) return LBM_OK;
  dev_free(c, *p);
  *p = nullptr;
  *cap = 0;
  const size_t n = std::max<size_t>(need + need / 2, 16);
  lbm_status st = dev_alloc(c, n * sizeof(T), (void**)p);
  if (st) return st;
  *cap = n;
  return LBM_OK;
}

template <typename T>
hipError_t put(lbm_ctx* c, T* dst, const std::vector<T>& v) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream);
}

std::string cache_key(const lbm_ctx* c) {
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) dev = prop.gcnArchName;
  for (auto& ch : dev)
    if (ch == '"' || ch == ':' || ch == ' ') ch = '_';
  std::ostringstream os;
  os << "Q" << c->Q << "_S" << c->storage << "_I" << c->n_inst << "_N" << c->total_nodes;
  if (c->n_inst == 1) os << "_" << c->desc[0].nx << "x" << c->desc[0].ny << "x" << c->desc[0].nz;
  os << "_" << dev;
  return os.str();
}

std::map<std::string, int> read_cache(const char* path) {
  std::map<std::string, int> m;
  if (!path) return m;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) continue;
    const size_t q1 = line.find('"', q0 + 1);
    const size_t colon = line.find(':', q1);
    if (q1 == std::string::npos || colon == std::string::npos) continue;
    m[line.substr(q0 + 1, q1 - q0 - 1)] = std::atoi(line.c_str() + colon + 1);
  }
  return m;
}

void write_cache(const char* path, const std::map<std::string, int>& m) {
  if (!path) return;
  std::ofstream out(path);
  out << "{\n";
  size_t k = 0;
  for (const auto& kv : m) out << "  \"" << kv.first << "\": " << kv.second << (++k < m.size() ? ",\n" : "\n");
  out << "}\n";
}

}  // namespace

extern "C" {

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID: return "invalid argument";
    case LBM_ERR_OOM: return "out of device memory";
    case LBM_ERR_DEVICE: return "device error";
    case LBM_ERR_NONFINITE: return "non-finite or invalid state";
    case LBM_ERR_GEOMETRY: return "body does not fit the domain";
    case LBM_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* lbm_last_error(const lbm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int lbm_variant_count(void) { return bulk_variant_count(); }
const char* lbm_variant_name(int v) { return bulk_variant_name(v); }

lbm_status lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  invalidate_graphs(c);
  dev_free(c, c->buf[0]);
  dev_free(c, c->buf[1]);
  dev_free(c, c->flags);
  dev_free(c, c->dinst);
  dev_free(c, c->dclock);
  dev_free(c, c->derr);
  dev_free(c, c->dneq_words);
  dev_free(c, c->dblist);
  dev_free(c, c->dbcount);
  dev_free(c, c->dtiles);
  dev_free(c, c->dregions);
  dev_free(c, c->dbtiles);
  dev_free(c, c->dgtiles);
  dev_free(c, c->dstats);
  dev_free(c, c->force_ws);
  dev_free(c, c->mp_field);
  for (auto& m : c->mesh) {
    dev_free(c, m.v);
    dev_free(c, m.f);
    dev_free(c, m.cs);
    dev_free(c, m.cx);
    dev_free(c, m.bs);
    dev_free(c, m.bf);
  }
  if (c->herr) (void)hipHostFree(c->herr);
  if (c->err_event) (void)hipEventDestroy(c->err_event);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return LBM_OK;
}

lbm_status lbm_create(const lbm_instance_desc* desc, int n_instances, const lbm_device_opts* opts,
                      lbm_ctx** out) {
  if (!out) return fail(nullptr, LBM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (!desc || n_instances < 1) return fail(nullptr, LBM_ERR_INVALID, "no instances");
  const int Q = desc[0].lattice, storage = desc[0].storage;
  for (int k = 0; k < n_instances; ++k) {
    const lbm_instance_desc& d = desc[k];
    if (d.lattice != LBM_D2Q9 && d.lattice != LBM_D3Q27)
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: unknown lattice %d", k, d.lattice);
    if (d.lattice != Q || d.storage != storage)
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: lattice/storage differ from instance 0", k);
    if (d.storage < LBM_F64 || d.storage > LBM_BF16_SHIFTED)
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: unknown storage %d", k, d.storage);
    if (d.nx < 1 || d.ny < 1 || d.nz < 1 || (Q == 9 && d.nz != 1))
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: bad sizes %dx%dx%d", k, d.nx, d.ny, d.nz);
    if ((int64_t)d.nx * d.ny * d.nz >= (int64_t(1) << 31))
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: more than 2^31 nodes", k);
    if (!(d.nu > 0.0) || !std::isfinite(d.nu))
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: nu must be > 0", k);
    if (d.collision != LBM_KBC && d.collision != LBM_LBGK)
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: unknown collision", k);
    if (!valid_faces(d)) return fail(nullptr, LBM_ERR_INVALID, "instance %d: invalid faces", k);
    if ((d.face[0] == LBM_FACE_INLET || d.face[1] == LBM_FACE_OUTLET) && d.nx < 2)
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: inflow / outflow faces need nx >= 2", k);
    if (d.inlet_profile != 0 && d.inlet_profile != 1)
      return fail(nullptr, LBM_ERR_INVALID, "instance %d: unknown inlet profile", k);
    if (d.ramp_steps < 0) return fail(nullptr, LBM_ERR_INVALID, "instance %d: ramp < 0", k);
    for (int a = 0; a < 3; ++a)
      if (!(std::fabs(d.u_in[a]) < 1.0)) return fail(nullptr, LBM_ERR_INVALID, "instance %d: |u_in| >= 1", k);
  }
  lbm_ctx* c = new lbm_ctx;
  c->Q = Q;
  c->D = Q == 27 ? 3 : 2;
  c->storage = storage;
  c->esize = storage_bytes(storage);
  c->ops = get_ops(Q, storage);
  c->n_inst = n_instances;
  c->desc.assign(desc, desc + n_instances);
  if (opts) {
    c->device = opts->device;
    c->ualloc = opts->alloc;
    c->ufree = opts->free;
    c->actx = opts->alloc_ctx;
    c->use_graph = opts->use_graph;
    if ((c->ualloc == nullptr) != (c->ufree == nullptr)) {
      delete c;
      return fail(nullptr, LBM_ERR_INVALID, "alloc and free callbacks must be given together");
    }
  }
  lbm_status st = LBM_OK;
  auto bail = [&](lbm_status s) {
    g_create_error = c->err;
    lbm_destroy(c);
    return s;
  };
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    fail(c, LBM_ERR_DEVICE, "hipSetDevice(%d) failed", c->device);
    return bail(LBM_ERR_DEVICE);
  }
  if (opts && opts->hip_stream) {
    c->stream = (hipStream_t)opts->hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      fail(c, LBM_ERR_DEVICE, "hipStreamCreate failed");
      return bail(LBM_ERR_DEVICE);
    }
    c->own_stream = true;
  }
  if ((st = resolve_scratch(c))) return bail(st);
  // Layout: per instance Q population arrays of stride round_up(N, 64).
  c->hinst.resize(n_instances);
  c->moving.assign(n_instances, 0);
  c->has_body.assign(n_instances, 0);
  c->has_faces.assign(n_instances, 0);
  c->mesh.assign(n_instances, lbm_ctx::MeshBuf());
  for (int k = 0; k < n_instances; ++k) {
    c->has_faces[k] = desc[k].face[0] == LBM_FACE_INLET || desc[k].face[1] == LBM_FACE_OUTLET;
    if (c->has_faces[k]) c->any_faces = true;
  }
  c->force_valid.assign(n_instances, 0);
  // Population arrays are padded so that consecutive arrays do not start a
  // power of two apart (which maps the Q loads of a wave onto the same HBM
  // channels); KBC_POP_PAD overrides the padding (elements, multiple of 64).
  int64_t pad = 0;
  if (const char* e = std::getenv("KBC_POP_PAD")) pad = std::max<int64_t>(0, std::atoll(e)) / 64 * 64;
  size_t off = 0, foff = 0;
  for (int k = 0; k < n_instances; ++k) {
    const lbm_instance_desc& d = desc[k];
    InstDev& I = c->hinst[k];
    std::memset(&I, 0, sizeof I);
    I.N = (int64_t)d.nx * d.ny * d.nz;
    I.stride = (I.N + 63) / 64 * 64 + pad;
    I.pop_off = (int64_t)off;
    off += (size_t)Q * I.stride;
    I.flag_off = needs_flags(d) ? (int64_t)foff : -1;
    foff += (size_t)((I.N + 255) / 256 * 256);
    I.nx = d.nx;
    I.ny = d.ny;
    I.nz = d.nz;
    I.D = c->D;
    I.divx = make_fastdiv((uint32_t)d.nx);
    I.divy = make_fastdiv((uint32_t)d.ny);
    I.beta = 1.0 / (6.0 * d.nu + 1.0);
    I.beta_f = (float)I.beta;
    I.near_eq = kNearEq;
    if (const char* e = std::getenv("KBC_NEAR_EQ")) I.near_eq = (float)std::atof(e);
    I.collision = d.collision;
    I.trace_in_s = d.kbc_trace_in_s ? 1 : 0;
    I.inlet_profile = d.inlet_profile;
    I.ramp_steps = d.ramp_steps;
    I.body_kind = LBM_BODY_NONE;
    for (int f = 0; f < 6; ++f) I.face[f] = d.face[f];
    for (int a = 0; a < 3; ++a) I.u_in[a] = d.u_in[a];
    c->total_nodes += I.N;
  }
  c->pop_elems = off;
  c->flag_bytes = foff;
  if ((st = dev_alloc(c, off * c->esize, &c->buf[0]))) return bail(st);
  if ((st = dev_alloc(c, off * c->esize, &c->buf[1]))) return bail(st);
  if ((st = dev_alloc(c, foff, (void**)&c->flags))) return bail(st);
  if ((st = dev_alloc(c, sizeof(int64_t), (void**)&c->dclock))) return bail(st);
  if ((st = dev_alloc(c, sizeof(uint32_t), (void**)&c->derr))) return bail(st);
  if ((st = dev_alloc(c, 2 * (size_t)(n_instances + 1) * sizeof(uint32_t), (void**)&c->dbcount))) return bail(st);
  if (hipHostMalloc((void**)&c->herr, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    fail(c, LBM_ERR_OOM, "hipHostMalloc failed");
    return bail(LBM_ERR_OOM);
  }
  *c->herr = 0;
  if (hipEventCreateWithFlags(&c->err_event, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
    fail(c, LBM_ERR_DEVICE, "hipEventCreate failed");
    return bail(LBM_ERR_DEVICE);
  }
  if (const char* e = std::getenv("KBC_SERIAL_BOUNDARY")) c->overlap = std::atoi(e) == 0;
  // Rest state: every deviation is zero in every storage format.
  if (hipMemsetAsync(c->buf[0], 0, off * c->esize, c->stream) != hipSuccess ||
      hipMemsetAsync(c->buf[1], 0, off * c->esize, c->stream) != hipSuccess ||
      hipMemsetAsync(c->flags, 0, foff, c->stream) != hipSuccess ||
      hipMemsetAsync(c->dclock, 0, sizeof(int64_t), c->stream) != hipSuccess ||
      hipMemsetAsync(c->derr, 0, sizeof(uint32_t), c->stream) != hipSuccess ||
      hipMemsetAsync(c->dbcount, 0, 2 * (size_t)(n_instances + 1) * sizeof(uint32_t), c->stream) != hipSuccess) {
    fail(c, LBM_ERR_DEVICE, "hipMemsetAsync failed");
    return bail(LBM_ERR_DEVICE);
  }
  // Static flags of non-periodic face planes (uploaded on the context's
  // stream, after the clears above; the host copies live until the final
  // synchronisation).
  std::vector<std::vector<uint8_t>> hflags(n_instances);
  for (int k = 0; k < n_instances; ++k) {
    const InstDev& I = c->hinst[k];
    if (I.flag_off < 0) continue;
    const lbm_instance_desc& d = desc[k];
    std::vector<uint8_t>& h = hflags[k];
    h.assign((size_t)I.N, 0);
    for (int z = 0; z < d.nz; ++z)
      for (int y = 0; y < d.ny; ++y)
        for (int x = 0; x < d.nx; ++x) {
          const int p[3] = {x, y, z}, n[3] = {d.nx, d.ny, d.nz};
          bool on = false;
          for (int a = 0; a < 3; ++a) {
            if (p[a] == 0 && d.face[2 * a] != LBM_FACE_PERIODIC) on = true;
            if (p[a] == n[a] - 1 && d.face[2 * a + 1] != LBM_FACE_PERIODIC) on = true;
          }
          if (on) h[(size_t)x + (size_t)d.nx * ((size_t)y + (size_t)d.ny * z)] = FLAG_STATIC;
        }
    if (hipMemcpyAsync(c->flags + I.flag_off, h.data(), h.size(), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess) {
      fail(c, LBM_ERR_DEVICE, "flag upload failed");
      return bail(LBM_ERR_DEVICE);
    }
  }
  if ((st = upload(c, &c->dinst, c->hinst))) return bail(st);
  if ((st = rebuild_tiles(c))) return bail(st);
  if ((st = rebuild_work(c))) return bail(st);
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    fail(c, LBM_ERR_DEVICE, "initial synchronisation failed");
    return bail(LBM_ERR_DEVICE);
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx* c, int inst, const double* rho, const double* u) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  if (!rho || !u) return fail(c, LBM_ERR_INVALID, "rho and u are required");
  const InstDev& I = c->hinst[inst];
  const int64_t N = I.N;
  for (int64_t n = 0; n < N; ++n) {
    if (!(rho[n] > 0.0) || !std::isfinite(rho[n])) return fail(c, LBM_ERR_INVALID, "rho <= 0 at node %lld", (long long)n);
    for (int a = 0; a < c->D; ++a)
      if (!(std::fabs(u[a * N + n]) < 1.0)) return fail(c, LBM_ERR_INVALID, "|u| >= 1 at node %lld", (long long)n);
  }
  double *dr = nullptr, *du = nullptr;
  if ((st = dev_alloc(c, N * sizeof(double), (void**)&dr))) return st;
  if ((st = dev_alloc(c, c->D * N * sizeof(double), (void**)&du))) {
    dev_free(c, dr);
    return st;
  }
  hipError_t e = hipMemcpyAsync(dr, rho, N * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(du, u, c->D * N * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = c->ops->init_eq(c->dinst, inst, N, dr, du, c->buf[c->cur], c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, dr);
  dev_free(c, du);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, "init_fields: %s", hipGetErrorString(e));
  c->force_valid[inst] = 0;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Surface-mesh body of instance inst: validates and copies the mesh, builds
// its column crossings and face cells on the host, uploads them, and points
// the instance descriptor at them.  A mesh replacing a mesh is the surface
// at the next step's time: the current geometry is kept and the next step
// refills what it uncovers; the swept box only grows (it covers the old
// and the new surface), and while it does not change, the descriptor is
// updated in place, so that captured graphs stay valid.
lbm_status set_mesh(lbm_ctx* c, int inst, const lbm_body& b) {
  const int D = c->D;
  if (b.nverts < (D == 3 ? 3 : 2) || b.ntris < 1 || !b.verts || !b.vert_vel || !b.tris)
    return fail(c, LBM_ERR_INVALID, "a mesh needs vertices, vertex velocities and faces");
  MeshHost m;
  m.v.assign(6 * (size_t)b.nverts, 0.0);
  for (int i = 0; i < b.nverts; ++i)
    for (int a = 0; a < 3; ++a) {
      const double x = a < D ? b.verts[3 * i + a] : 0.0;
      const double v = a < D ? b.vert_vel[3 * i + a] : 0.0;
      if (!std::isfinite(x) || !std::isfinite(v) || !(std::fabs(v) < 1.0))
        return fail(c, LBM_ERR_INVALID, "mesh vertex %d: non-finite coordinate or |velocity| >= 1", i);
      m.v[3 * (size_t)i + a] = x;
      m.v[3 * (size_t)b.nverts + 3 * (size_t)i + a] = v;
    }
  m.f.assign(b.tris, b.tris + 3 * (size_t)b.ntris);
  for (size_t k = 0; k < m.f.size(); ++k) {
    if (D == 2 && k % 3 == 2) m.f[k] = m.f[k - 2];   // unused in 2D
    if (m.f[k] < 0 || m.f[k] >= b.nverts)
      return fail(c, LBM_ERR_INVALID, "mesh face %zu: vertex index out of range", k / 3);
  }
  // Swept box: the surface's bounding box with a 2-node margin (as for the
  // analytic bodies), joined with the previous box when a mesh replaces a
  // mesh.
  const lbm_instance_desc& d = c->desc[inst];
  const int n[3] = {d.nx, d.ny, d.nz};
  InstDev& I = c->hinst[inst];
  const bool was_mesh = I.body_kind == LBM_BODY_MESH;
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= D) {
      lo[a] = 0;
      hi[a] = 1;
      continue;
    }
    double mn = 1e300, mx = -1e300;
    for (int i = 0; i < b.nverts; ++i) {
      mn = std::min(mn, m.v[3 * (size_t)i + a]);
      mx = std::max(mx, m.v[3 * (size_t)i + a]);
    }
    int l = (int)std::floor(mn) - 2, h = (int)std::ceil(mx) + 3;
    if (was_mesh) {
      l = std::min(l, I.box_lo[a]);
      h = std::max(h, I.box_hi[a]);
    }
    if (l < 0 || h > n[a]) {
      if (d.face[2 * a] == LBM_FACE_PERIODIC)
        return fail(c, LBM_ERR_GEOMETRY, "the mesh's swept region crosses a periodic face");
      l = std::max(l, 0);
      h = std::min(h, n[a]);
    }
    if (h <= l) return fail(c, LBM_ERR_GEOMETRY, "the mesh lies outside the domain");
    lo[a] = l;
    hi[a] = h;
  }
  mesh_columns(D, lo, hi, m);
  mesh_cells(D, m);
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  lbm_ctx::MeshBuf& mb = c->mesh[inst];
  lbm_status st;
  if ((st = ensure_dev(c, &mb.v, &mb.v_cap, m.v.size()))) return st;
  if ((st = ensure_dev(c, &mb.f, &mb.f_cap, m.f.size()))) return st;
  if ((st = ensure_dev(c, &mb.cs, &mb.cs_cap, m.cs.size()))) return st;
  if ((st = ensure_dev(c, &mb.cx, &mb.cx_cap, std::max<size_t>(m.cx.size(), 1)))) return st;
  if ((st = ensure_dev(c, &mb.bs, &mb.bs_cap, m.bs.size()))) return st;
  if ((st = ensure_dev(c, &mb.bf, &mb.bf_cap, std::max<size_t>(m.bf.size(), 1)))) return st;
  hipError_t e = put(c, mb.v, m.v);
  if (e == hipSuccess) e = put(c, mb.f, m.f);
  if (e == hipSuccess) e = put(c, mb.cs, m.cs);
  if (e == hipSuccess) e = put(c, mb.cx, m.cx);
  if (e == hipSuccess) e = put(c, mb.bs, m.bs);
  if (e == hipSuccess) e = put(c, mb.bf, m.bf);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, "mesh upload: %s", hipGetErrorString(e));
  if (I.flag_off < 0) {
    int64_t foff = 0;
    for (int k = 0; k < inst; ++k) foff += (c->hinst[k].N + 255) / 256 * 256;
    I.flag_off = foff;
  }
  const bool same_box = was_mesh && std::equal(lo, lo + 3, I.box_lo) && std::equal(hi, hi + 3, I.box_hi);
  I.body_kind = LBM_BODY_MESH;
  for (int k = 0; k < 16; ++k) I.body[k] = 0.0;
  for (int a = 0; a < 3; ++a) {
    I.box_lo[a] = lo[a];
    I.box_hi[a] = hi[a];
  }
  I.mesh_v = mb.v;
  I.mesh_vel = mb.v + 3 * (size_t)b.nverts;
  I.mesh_f = mb.f;
  I.mesh_nf = b.ntris;
  I.col_start = mb.cs;
  I.col_x = mb.cx;
  I.bin_start = mb.bs;
  I.bin_face = mb.bf;
  for (int a = 0; a < 2; ++a) {
    I.col_lo[a] = m.col_lo[a];
    I.col_n[a] = m.col_n[a];
  }
  for (int a = 0; a < 3; ++a) {
    I.bin_lo[a] = m.bin_lo[a];
    I.bin_n[a] = m.bin_n[a];
  }
  I.bin_h = m.bin_h;
  c->has_body[inst] = 1;
  c->moving[inst] = 1;   // the geometry stages read the mesh every step
  c->force_valid[inst] = 0;
  if (same_box) {
    // Descriptor contents only: the device copy keeps its address.
    HIPCHECK(c, hipMemcpyAsync(c->dinst, c->hinst.data(), c->hinst.size() * sizeof(InstDev),
                               hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
  }
  if ((st = upload(c, &c->dinst, c->hinst))) return st;
  HIPCHECK(c, hipMemcpyAsync(c->dclock, &c->step, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  if (!was_mesh && (st = full_geometry(c, inst))) return st;
  return rebuild_work(c);
}

}  // namespace

extern "C" {

lbm_status lbm_set_geometry(lbm_ctx* c, int inst, const lbm_body* body) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  lbm_body b;
  std::memset(&b, 0, sizeof b);
  if (body) b = *body;
  if (b.kind < LBM_BODY_NONE || b.kind > LBM_BODY_PLATES)
    return fail(c, LBM_ERR_INVALID, "unknown body kind %d", b.kind);
  if (b.kind == LBM_BODY_MESH) return set_mesh(c, inst, b);
  if (b.kind == LBM_BODY_FLAP && c->D != 2) return fail(c, LBM_ERR_INVALID, "flap bodies are 2D only");
  for (int k = 0; k < 16; ++k)
    if (!std::isfinite(b.params[k])) return fail(c, LBM_ERR_INVALID, "non-finite body parameter");
  if (b.kind == LBM_BODY_SPHERE && !(b.params[3] > 0.0)) return fail(c, LBM_ERR_INVALID, "radius must be > 0");
  if (b.kind == LBM_BODY_FLAP && !(b.params[1] > 0.0 && b.params[2] > 0.0))
    return fail(c, LBM_ERR_INVALID, "flap length and thickness must be > 0");
  InstDev& I = c->hinst[inst];
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  if (b.kind != LBM_BODY_NONE && !body_box(c, inst, b, lo, hi))
    return fail(c, LBM_ERR_GEOMETRY, "the body's swept region crosses a periodic face");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  if (I.flag_off < 0) {
    // Instance had no flags yet: its slice of the pool is zero already.
    int64_t foff = 0;
    for (int k = 0; k < inst; ++k) foff += (c->hinst[k].N + 255) / 256 * 256;
    I.flag_off = foff;
  }
  I.body_kind = b.kind;
  for (int k = 0; k < 16; ++k) I.body[k] = b.params[k];
  for (int a = 0; a < 3; ++a) {
    I.box_lo[a] = lo[a];
    I.box_hi[a] = hi[a];
  }
  const double* p = b.params;
  c->has_body[inst] = b.kind != LBM_BODY_NONE;
  c->moving[inst] = (b.kind == LBM_BODY_SPHERE && p[7] != 0.0 && (p[4] != 0.0 || p[5] != 0.0 || p[6] != 0.0)) ||
                    (b.kind == LBM_BODY_FLAP && p[4] != 0.0 && p[3] != 0.0);
  if ((st = upload(c, &c->dinst, c->hinst))) return st;
  HIPCHECK(c, hipMemcpyAsync(c->dclock, &c->step, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  if ((st = full_geometry(c, inst))) return st;
  if ((st = rebuild_work(c))) return st;
  c->force_valid[inst] = 0;
  return LBM_OK;
}

lbm_status lbm_set_multiphase(lbm_ctx* c, int inst, int enable, double kappa, double kappa_w) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  if (enable) {
    if (c->storage != LBM_F64 && c->storage != LBM_F32)
      return fail(c, LBM_ERR_UNSUPPORTED, "multiphase needs FP64 or FP32 storage");
    if (!std::isfinite(kappa) || !std::isfinite(kappa_w))
      return fail(c, LBM_ERR_INVALID, "non-finite multiphase coefficient");
    for (int k = 0; k < 6; ++k)
      if (c->hinst[inst].face[k] != LBM_FACE_PERIODIC && c->hinst[inst].face[k] != LBM_FACE_WALL)
        return fail(c, LBM_ERR_UNSUPPORTED, "multiphase needs periodic or wall faces");
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const size_t fsz = c->storage == LBM_F64 ? sizeof(double) : sizeof(float);
  if (enable && !c->mp_field) {
    if ((st = dev_alloc(c, 3 * (size_t)c->total_nodes * fsz, &c->mp_field))) return st;
    HIPCHECK(c, hipMemsetAsync(c->mp_field, 0, 3 * (size_t)c->total_nodes * fsz, c->stream));
  }
  InstDev& I = c->hinst[inst];
  I.mp = enable ? 1 : 0;
  I.mp_kappa = enable ? kappa : 0.0;
  I.mp_kappa_w = enable ? kappa_w : 0.0;
  bool any = false;
  for (int k = 0; k < c->n_inst; ++k) any = any || c->hinst[k].mp;
  int64_t off = 0;
  for (int k = 0; k < c->n_inst; ++k) {
    c->hinst[k].mp_field = any ? static_cast<char*>(c->mp_field) + 3 * (size_t)off * fsz : nullptr;
    off += c->hinst[k].N;
  }
  c->any_mp = any;
  if ((st = upload(c, &c->dinst, c->hinst))) return st;
  invalidate_graphs(c);
  c->force_valid[inst] = 0;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int n_steps) {
  if (!c) return LBM_ERR_INVALID;
  if (n_steps < 0) return fail(c, LBM_ERR_INVALID, "n_steps < 0");
  if (c->err_pending && hipEventQuery(c->err_event) == hipSuccess) {
    c->err_pending = false;
    if (*c->herr) return fail(c, LBM_ERR_NONFINITE, "a node reached an invalid state");
  }
  lbm_status st;
  int n = n_steps;
  while (n > 0) {
    if (c->use_graph && n >= 2 && !c->graph_failed) {
      if ((st = ensure_graph(c, c->cur))) return st;
      if (c->graph[c->cur]) {
        HIPCHECK(c, hipGraphLaunch(c->graph[c->cur], c->stream));
        n -= 2;
        c->step += 2;
        continue;
      }
    }
    if ((st = enqueue_step(c, c->cur))) return st;
    c->cur ^= 1;
    c->step += 1;
    n -= 1;
  }
  if (n_steps > 0) {
    for (int k = 0; k < c->n_inst; ++k) c->force_valid[k] = 1;
    if (!c->err_pending) {
      HIPCHECK(c, hipMemcpyAsync(c->herr, c->derr, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream));
      HIPCHECK(c, hipEventRecord(c->err_event, c->stream));
      c->err_pending = true;
    }
  }
  return LBM_OK;
}

lbm_status lbm_synchronize(lbm_ctx* c) {
  if (!c) return LBM_ERR_INVALID;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return check_error_word(c);
}

lbm_status lbm_moments(lbm_ctx* c, int inst, double* rho, double* u, lbm_totals* tot) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const InstDev& I = c->hinst[inst];
  const int64_t N = I.N;
  double *dr = nullptr, *du = nullptr, *dp = nullptr, *dout = nullptr;
  const int64_t nparts_max = (N + 255) / 256;
  if ((st = dev_alloc(c, N * sizeof(double), (void**)&dr))) return st;
  if ((st = dev_alloc(c, c->D * N * sizeof(double), (void**)&du))) { dev_free(c, dr); return st; }
  if ((st = dev_alloc(c, nparts_max * 4 * sizeof(double) + 64 * sizeof(double), (void**)&dp))) {
    dev_free(c, dr); dev_free(c, du); return st;
  }
  dout = dp + nparts_max * 4;
  int np = 0;
  hipError_t e = c->ops->moments(c->dinst, inst, N, c->buf[c->cur], c->flags, dr, du, dp, &np, c->stream);
  if (e == hipSuccess) e = launch_reduce(dp, np, 4, dout, c->stream);
  double sums[4] = {0, 0, 0, 0};
  StatPartial sp[3];
  bool have_stats = false;
  if (e == hipSuccess && tot && c->stats_enabled && c->step > 0) {
    StatPartial* so = reinterpret_cast<StatPartial*>(dout + 8);
    e = launch_reduce_stats(c->dstats + c->tile_first[inst], c->tile_count[inst], so, c->stream);
    // The boundary and FP64 passes serve all instances at once; their nodes
    // are attributed to the instance only in single-instance contexts.
    if (e == hipSuccess)
      e = launch_reduce_stats(c->dstats + c->tiles.size(), c->n_inst == 1 ? c->bstat_slots : 0,
                              so + 1, c->stream);
    if (e == hipSuccess)
      e = launch_reduce_stats(c->dstats + c->tiles.size() + c->bstat_slots,
                              c->n_inst == 1 ? kFixupBlocks : 0, so + 2, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(sp, so, sizeof sp, hipMemcpyDeviceToHost, c->stream);
    have_stats = true;
  }
  if (e == hipSuccess) e = hipMemcpyAsync(sums, dout, sizeof sums, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && rho) e = hipMemcpyAsync(rho, dr, N * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && u) e = hipMemcpyAsync(u, du, c->D * N * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, dr);
  dev_free(c, du);
  dev_free(c, dp);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, "moments: %s", hipGetErrorString(e));
  if (tot) {
    std::memset(tot, 0, sizeof *tot);
    tot->mass = sums[0];
    for (int a = 0; a < 3; ++a) tot->momentum[a] = sums[1 + a];
    tot->gamma_min = tot->gamma_mean = tot->gamma_max = 2.0;
    if (have_stats) {
      uint64_t cnt = 0, f64 = 0;
      double gsum = 0.0;
      float gmin = 1e30f, gmax = -1e30f;
      for (int k = 0; k < 3; ++k) {
        if (!sp[k].count) continue;
        cnt += sp[k].count;
        f64 += sp[k].fp64;
        gsum += sp[k].gsum;
        gmin = std::min(gmin, sp[k].gmin);
        gmax = std::max(gmax, sp[k].gmax);
      }
      if (cnt) {
        tot->gamma_min = gmin;
        tot->gamma_max = gmax;
        tot->gamma_mean = gsum / (double)cnt;
        tot->fp64_gamma_fraction = (double)f64 / (double)cnt;
      }
    }
    tot->step = c->step;
  }
  return check_error_word(c);
}

}  // extern "C"

namespace {

// Doubles of wall-force workspace for n_q points: points, normals, weights,
// tractions, partial sums, reduced sums.
size_t force_ws_need(const lbm_ctx* c, int n_q) {
  const size_t np = (size_t)(n_q + force_points_per_workgroup(c->Q) - 1) /
                    (size_t)force_points_per_workgroup(c->Q);
  return (size_t)n_q * (3 * c->D + 1) + np * 4 + 8;
}

// Wall force through the workspace ws (force_ws_need doubles): uploads the points,
// runs the force kernel and the fixed-order reduction on the context stream,
// copies the results out.  No allocation.
lbm_status wall_force_run(lbm_ctx* c, int inst, const double* xq, const double* nq,
                          const double* wq, int n_q, double* traction, double force[3],
                          double* ws) {
  const int D = c->D;
  const size_t np_max = (size_t)(n_q + force_points_per_workgroup(c->Q) - 1) /
                        (size_t)force_points_per_workgroup(c->Q);
  double *dx = ws, *dn = dx + (size_t)n_q * D, *dw = dn + (size_t)n_q * D, *dt = dw + n_q;
  double *dp = dt + (size_t)n_q * D, *dout = dp + np_max * 4;
  int np = 0;
  double sums[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(dx, xq, (size_t)n_q * D * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dn, nq, (size_t)n_q * D * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dw, wq, (size_t)n_q * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = c->ops->force(c->dinst, inst, c->buf[1 - c->cur], c->flags, c->dclock, dx, dn, dw, n_q, dt,
                      dp, &np, c->stream);
  if (e == hipSuccess) e = launch_reduce(dp, np, 4, dout, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(sums, dout, sizeof sums, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && traction)
    e = hipMemcpyAsync(traction, dt, (size_t)n_q * D * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, "wall force: %s", hipGetErrorString(e));
  for (int a = 0; a < D; ++a) force[a] = sums[a];
  if (sums[3] != 0.0)
    return fail(c, LBM_ERR_GEOMETRY, "%d probes found no fluid node within two spacings", (int)sums[3]);
  return LBM_OK;
}

lbm_status wall_force_args(lbm_ctx* c, int inst, const double* xq, const double* nq,
                           const double* wq, int n_q, double force[3]) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  if (!force || n_q < 0 || (n_q > 0 && (!xq || !nq || !wq)))
    return fail(c, LBM_ERR_INVALID, "bad quadrature arguments");
  if (!c->force_valid[inst])
    return fail(c, LBM_ERR_INVALID, "wall force needs a step after the last geometry or state change");
  if (c->hinst[inst].mp)
    return fail(c, LBM_ERR_UNSUPPORTED, "no wall force for a multiphase instance");
  force[0] = force[1] = force[2] = 0.0;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_wall_force(lbm_ctx* c, int inst, const double* xq, const double* nq,
                          const double* wq, int n_q, double* traction, double force[3]) {
  lbm_status st = wall_force_args(c, inst, xq, nq, wq, n_q, force);
  if (st || n_q == 0) return st;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  // The workspace persists across calls and grows only for a larger n_q.
  const size_t need = force_ws_need(c, n_q);
  if (need > c->force_ws_doubles) {
    dev_free(c, c->force_ws);
    c->force_ws = nullptr;
    c->force_ws_doubles = 0;
    if ((st = dev_alloc(c, need * sizeof(double), (void**)&c->force_ws))) return st;
    c->force_ws_doubles = need;
  }
  return wall_force_run(c, inst, xq, nq, wq, n_q, traction, force, c->force_ws);
}

lbm_status lbm_wall_force_noalloc(lbm_ctx* c, int inst, const double* xq, const double* nq,
                                  const double* wq, int n_q, double* traction, double force[3]) {
  lbm_status st = wall_force_args(c, inst, xq, nq, wq, n_q, force);
  if (st || n_q == 0) return st;
  if (n_q > kNoAllocMaxPoints)
    return fail(c, LBM_ERR_INVALID, "n_q = %d exceeds the %d points of the static workspace", n_q,
                kNoAllocMaxPoints);
  if (force_ws_need(c, n_q) > kForceScratchDoubles)
    return fail(c, LBM_ERR_INVALID, "static workspace too small for n_q = %d", n_q);
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  return wall_force_run(c, inst, xq, nq, wq, n_q, traction, force, c->scratch);
}

lbm_status lbm_get_populations(lbm_ctx* c, int inst, double* f) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  if (!f) return fail(c, LBM_ERR_INVALID, "f is NULL");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const int64_t N = c->hinst[inst].N;
  double* df = nullptr;
  if ((st = dev_alloc(c, (size_t)c->Q * N * sizeof(double), (void**)&df))) return st;
  hipError_t e = c->ops->decode(c->dinst, inst, N, c->buf[c->cur], df, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f, df, (size_t)c->Q * N * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, df);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, "get_populations: %s", hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_get_populations_box(lbm_ctx* c, int inst, const int lo[3], const int hi[3],
                                   double* f) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  if (!f || !lo || !hi) return fail(c, LBM_ERR_INVALID, "f, lo and hi are required");
  const lbm_instance_desc& d = c->desc[inst];
  const int n[3] = {d.nx, d.ny, d.nz};
  int ext[3];
  for (int a = 0; a < 3; ++a) {
    ext[a] = hi[a] - lo[a];
    const bool periodic = d.face[2 * a] == LBM_FACE_PERIODIC;
    const bool ok = ext[a] >= 1 && (periodic ? (lo[a] >= -n[a] && hi[a] <= 2 * n[a] && ext[a] <= n[a])
                                             : (lo[a] >= 0 && hi[a] <= n[a]));
    if (!ok) return fail(c, LBM_ERR_INVALID, "box [%d, %d) invalid along axis %d", lo[a], hi[a], a);
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const int64_t Nb = (int64_t)ext[0] * ext[1] * ext[2];
  double* df = nullptr;
  if ((st = dev_alloc(c, (size_t)c->Q * Nb * sizeof(double), (void**)&df))) return st;
  hipError_t e = c->ops->decode_box(c->dinst, inst, lo, ext, c->buf[c->cur], df, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(f, df, (size_t)c->Q * Nb * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, df);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, "get_populations_box: %s", hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, int inst, const double* f) {
  lbm_status st = check_inst(c, inst);
  if (st) return st;
  if (!f) return fail(c, LBM_ERR_INVALID, "f is NULL");
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  const int64_t N = c->hinst[inst].N;
  double* df = nullptr;
  if ((st = dev_alloc(c, (size_t)c->Q * N * sizeof(double), (void**)&df))) return st;
  hipError_t e = hipMemcpyAsync(df, f, (size_t)c->Q * N * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = c->ops->encode(c->dinst, inst, N, df, c->buf[c->cur], c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  dev_free(c, df);
  if (e != hipSuccess) return fail(c, LBM_ERR_DEVICE, "set_populations: %s", hipGetErrorString(e));
  c->force_valid[inst] = 0;
  return LBM_OK;
}

lbm_status lbm_set_stats(lbm_ctx* c, int enabled) {
  if (!c) return LBM_ERR_INVALID;
  if ((enabled != 0) != (c->stats_enabled != 0)) invalidate_graphs(c);
  c->stats_enabled = enabled != 0;
  return LBM_OK;
}

lbm_status lbm_set_launch_mode(lbm_ctx* c, int mode) {
  if (!c) return LBM_ERR_INVALID;
  if (mode != 0 && mode != 1) return fail(c, LBM_ERR_INVALID, "launch mode must be 0 or 1");
  if (mode != c->launch_mode) invalidate_graphs(c);
  c->launch_mode = mode;
  return LBM_OK;
}

// Whether every instance's population arrays fit in a 4 GiB window.
static bool fits_off32(const lbm_ctx* c) {
  for (const InstDev& I : c->hinst)
    if ((uint64_t)c->Q * (uint64_t)I.stride * (uint64_t)c->esize >= (uint64_t(1) << 32)) return false;
  return true;
}

lbm_status lbm_set_variant(lbm_ctx* c, int v) {
  if (!c) return LBM_ERR_INVALID;
  if (v < 0 || v >= bulk_variant_count()) return fail(c, LBM_ERR_INVALID, "variant %d out of range", v);
  if (bulk_variant_off32(v) && !fits_off32(c))
    return fail(c, LBM_ERR_UNSUPPORTED, "variant %s needs instances below 4 GiB of populations",
                bulk_variant_name(v));
  if (v == c->variant) return LBM_OK;
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  c->variant = v;
  return rebuild_tiles(c);
}

lbm_status lbm_autotune(lbm_ctx* c, const char* cache_path, int* chosen) {
  if (!c) return LBM_ERR_INVALID;
  const std::string key = cache_key(c);
  std::map<std::string, int> cache = read_cache(cache_path);
  auto it = cache.find(key);
  lbm_status st;
  if (it != cache.end() && it->second >= 0 && it->second < bulk_variant_count()) {
    if ((st = lbm_set_variant(c, it->second))) return st;
    if (chosen) *chosen = c->variant;
    return LBM_OK;
  }
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  // Save both population buffers, flags and clock; the trial steps are undone
  // afterwards.  The other buffer matters too: nodes inside a moving body are
  // never written while solid, so they keep what was last stored there, and a
  // trial run moves the body further than the caller has.
  const size_t pbytes = c->pop_elems * c->esize;
  char* save = nullptr;
  uint8_t* fsave = nullptr;
  if ((st = dev_alloc(c, 2 * pbytes, (void**)&save))) return st;
  if ((st = dev_alloc(c, c->flag_bytes, (void**)&fsave))) { dev_free(c, save); return st; }
  const int cur0 = c->cur;
  HIPCHECK(c, hipMemcpyAsync(save, c->buf[cur0], pbytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHECK(c, hipMemcpyAsync(save + pbytes, c->buf[1 - cur0], pbytes, hipMemcpyDeviceToDevice,
                             c->stream));
  HIPCHECK(c, hipMemcpyAsync(fsave, c->flags, c->flag_bytes, hipMemcpyDeviceToDevice, c->stream));
  const int64_t step0 = c->step;
  hipEvent_t e0, e1;
  HIPCHECK(c, hipEventCreate(&e0));
  HIPCHECK(c, hipEventCreate(&e1));
  int best = c->variant;
  float best_ms = 1e30f;
  for (int v = 0; v < bulk_variant_count(); ++v) {
    if (bulk_variant_off32(v) && !fits_off32(c)) continue;
    if ((st = lbm_set_variant(c, v))) break;
    // Every candidate starts from the saved state, so that all are timed on
    // the same flow (a developing flow changes the boundary and FP64 work).
    HIPCHECK(c, hipMemcpyAsync(c->buf[cur0], save, pbytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->flags, fsave, c->flag_bytes, hipMemcpyDeviceToDevice, c->stream));
    HIPCHECK(c, hipMemcpyAsync(c->dclock, &step0, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    c->cur = cur0;
    c->step = step0;
    if ((st = lbm_step(c, 2))) break;
    HIPCHECK(c, hipEventRecord(e0, c->stream));
    if ((st = lbm_step(c, 16))) break;
    HIPCHECK(c, hipEventRecord(e1, c->stream));
    HIPCHECK(c, hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHECK(c, hipEventElapsedTime(&ms, e0, e1));
    if (ms < best_ms) {
      best_ms = ms;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHECK(c, hipMemcpyAsync(c->buf[cur0], save, pbytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHECK(c, hipMemcpyAsync(c->buf[1 - cur0], save + pbytes, pbytes, hipMemcpyDeviceToDevice,
                             c->stream));
  HIPCHECK(c, hipMemcpyAsync(c->flags, fsave, c->flag_bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHECK(c, hipMemcpyAsync(c->dclock, &step0, sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  HIPCHECK(c, hipMemsetAsync(c->derr, 0, sizeof(uint32_t), c->stream));
  HIPCHECK(c, hipStreamSynchronize(c->stream));
  dev_free(c, save);
  dev_free(c, fsave);
  c->cur = cur0;
  c->step = step0;
  c->err_pending = false;
  for (int k = 0; k < c->n_inst; ++k) c->force_valid[k] = 0;
  if (st) return st;
  if ((st = lbm_set_variant(c, best))) return st;
  cache[key] = best;
  write_cache(cache_path, cache);
  if (chosen) *chosen = best;
  return LBM_OK;
}

lbm_status lbm_info(const lbm_ctx* c, int inst, int64_t* nodes, int64_t* total_nodes,
                    int* bytes_per_update, int64_t* step) {
  if (!c) return LBM_ERR_INVALID;
  if (inst < 0 || inst >= c->n_inst) return LBM_ERR_INVALID;
  if (nodes) *nodes = c->hinst[inst].N;
  if (total_nodes) *total_nodes = c->total_nodes;
  if (bytes_per_update) *bytes_per_update = 2 * c->Q * c->esize;
  if (step) *step = c->step;
  return LBM_OK;
}

}  // extern "C"
