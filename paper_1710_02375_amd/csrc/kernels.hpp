// Launch interface between the host engine and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.hpp"

namespace kbc {

// Per-workgroup gamma statistics of one step.
struct StatPartial {
  float gmin, gmax;
  double gsum;
  uint32_t count, fp64;
};

// A run of nodes of one scanned box (boundary and geometry kernels).
struct BoxTile {
  int region;     // index into the region table
  int count;
  int64_t local0; // first node index inside the box, x-fastest
};

struct StepBuffers {
  const InstDev* insts;
  const void* src;
  void* dst;
  const uint8_t* flags;   // flag pool (instance offsets in InstDev)
  uint32_t* err;          // device error word
  const int64_t* clock;   // steps taken before this step
  StatPartial* stats;     // per-workgroup statistics, or null
  // Near-equilibrium nodes deferred to the FP64 pass: one 64-bit mask per
  // 64 consecutive nodes of a tile, word ti * neq_wpt + j for nodes
  // [64 j, 64 j + 64) of tile ti (neq_wpt = tile size / 64), bit l for the
  // node 64 j + l.  Every word is zero at the start of a step; the bulk
  // kernel stores the words with a deferred node, and the FP64 pass reads
  // neq_nwords words (none in the multiphase pipeline) and clears those set.
  uint64_t* neq_words;
  uint32_t neq_nwords;
  uint32_t neq_wpt;
  const Tile* tiles;      // the tile table the bulk kernel ran over
  int64_t* clock_tick;    // advanced by one at the end of the step, or null
  uint32_t* bcount;       // boundary-list counters, cleared by the FP64 pass
  int nbcount;
};

struct Ops {
  // Bulk stream-collide over tiles [tile0, tile0 + ntiles) for nodes with no
  // special flag, and the inflow / outflow plane nodes of those tiles.
  // Statistics go to stats[tile index].
  // faces: some instance of the launch has an inflow or outflow face; the
  // kernel then also forms the equilibria of those plane nodes (after its
  // main loop), otherwise the instantiation without that loop runs.
  hipError_t (*bulk)(int variant, const StepBuffers& b, const Tile* tiles, int tile0, int ntiles,
                     bool faces, hipStream_t s);
  // Nodes with missing populations of the scanned box tiles [bt0, bt0+nbt):
  // a scan appends the nodes with a cut link to a body to list[0, cap)
  // through count[0] and the nodes whose missing populations all come from
  // wall faces to list[cap, 2 cap) through count[1]; then nwg one-wavefront
  // workgroups fill and collide the first (one node per wavefront in 3D, two
  // in 2D) and nwall workgroups of 64 threads the second (one node per
  // thread).  Inflow and outflow plane nodes are handled by the bulk kernel.
  // Either workgroup count may be zero (no body, no wall face): that kernel
  // is not launched.  Both counts must be zero on entry (the FP64 pass
  // clears them).  Statistics go to stats[stat0, stat0 + nwg + nwall).
  hipError_t (*boundary)(const StepBuffers& b, const Region* regions, const BoxTile* btiles,
                         int bt0, int nbt, uint2* list, uint32_t cap, uint32_t* count, int nwg,
                         int nwall, int stat0, bool pre, hipStream_t s);
  // Geometry update over the swept boxes at time clock + toff: stage 0 marks
  // SOLID_NEXT and refills the fresh nodes of src, stage 1 does nothing (kept
  // for the call sequence), stage 2 makes SOLID_NEXT current and marks the
  // cut-link (BODY) nodes.
  hipError_t (*geometry)(int stage, const InstDev* insts, const Region* regions,
                         const BoxTile* gtiles, int ngt, void* src, uint8_t* flags,
                         const int64_t* clock, int toff, hipStream_t s);
  // f := f^eq(rho, u) on every node of one instance (rho: N, u: D*N doubles).
  hipError_t (*init_eq)(const InstDev* insts, int inst, int64_t N, const double* rho,
                        const double* u, void* buf, hipStream_t s);
  // Full populations (double, population-major) <-> storage.
  hipError_t (*decode)(const InstDev* insts, int inst, int64_t N, const void* buf, double* f,
                       hipStream_t s);
  hipError_t (*encode)(const InstDev* insts, int inst, int64_t N, const double* f, void* buf,
                       hipStream_t s);
  // rho, u (nullable) and per-workgroup partial sums (mass, momentum) of one
  // instance; returns the number of partials written through nparts.
  hipError_t (*moments)(const InstDev* insts, int inst, int64_t N, const void* buf,
                        const uint8_t* flags, double* rho, double* u, double* partials,
                        int* nparts, hipStream_t s);
  // Redoes the deferred near-equilibrium nodes with the FP64 gamma (grid of
  // nblocks workgroups striding over the mask words); statistics go to
  // stats[stat0 + workgroup].  It also ends the step: clears the boundary
  // list counters and advances clock_tick.
  hipError_t (*fixup)(const StepBuffers& b, int nblocks, int stat0, hipStream_t s);
  // Wall force (per point traction, per-workgroup partial force sums: four
  // doubles per workgroup, force_points_per_workgroup(Q) points each).
  hipError_t (*force)(const InstDev* insts, int inst, const void* prev, const uint8_t* flags,
                      const int64_t* clock, const double* xq, const double* nq,
                      const double* wq, int nqp, double* traction, double* partials,
                      int* nparts, hipStream_t s);
  // Full populations of the box [lo, lo + ext) (x-fastest, population-major).
  hipError_t (*decode_box)(const InstDev* insts, int inst, const int* lo, const int* ext,
                           const void* buf, double* f, hipStream_t s);
  // Multiphase step passes over tiles (Sec. III.B): stage 0 streams the nodes
  // with no special flag into dst and fills the density and phi fields,
  // stage 1 the density Laplacian, stage 2 forms the body force and the
  // forced collision of every fluid node in place.  Run after the boundary
  // launch in its pre-collision mode (pre = true: the boundary kernels write
  // the pre-collision state and density of their nodes instead of
  // colliding).
  hipError_t (*mp)(int stage, const StepBuffers& b, const Tile* tiles, int tile0, int ntiles,
                   hipStream_t s);
};

const Ops* get_ops(int Q, int storage);

// Boundary nodes handled by one workgroup (wavefront) at a time.
int boundary_nodes_per_workgroup(int Q);

// Quadrature points per workgroup of the wall-force kernel (its partial-sum
// count is ceil(n_q / this)).
int force_points_per_workgroup(int Q);

// Bulk-kernel variants (workgroup size, nodes per tile, waves per SIMD hint).
int bulk_variant_count();
const char* bulk_variant_name(int v);
int bulk_variant_tile(int v);
// True if the variant addresses populations with 32-bit byte offsets from one
// base per instance (requires Q * stride * sizeof(storage) < 2^32).
bool bulk_variant_off32(int v);

// Sums `width` doubles over n partials in a fixed order into out[width].
hipError_t launch_reduce(const double* partials, int n, int width, double* out, hipStream_t s);
hipError_t launch_reduce_stats(const StatPartial* parts, int n, StatPartial* out, hipStream_t s);

}  // namespace kbc
