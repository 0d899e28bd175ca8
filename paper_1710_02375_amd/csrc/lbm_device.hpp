// Device-side building blocks of the KBC lattice Boltzmann library for gfx950:
// lattice constants, population storage formats, fast integer division and the
// per-instance descriptor the kernels read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace kbc {

// ---------------------------------------------------------------------------
// Lattice: tensor product of D1Q3, velocity index i = (cx+1) + 3(cy+1) + 9(cz+1).
// Weights W_i are "lattice-specific constants" (Sec. II.A); the D1Q3 weights
// 2/3, 1/6, 1/6 give the speed of sound 1/sqrt(3) of Eq. 7.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int cx(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
template <int Q>
__host__ __device__ constexpr int cz(int i) { return Q == 27 ? i / 9 - 1 : 0; }
template <int Q>
__host__ __device__ constexpr int dims() { return Q == 27 ? 3 : 2; }
template <int Q>
__host__ __device__ constexpr int rest() { return (Q - 1) / 2; }
__host__ __device__ constexpr double w1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
template <int Q>
__host__ __device__ constexpr double weight(int i) {
  return w1d(cx(i)) * w1d(cy(i)) * (Q == 27 ? w1d(cz<Q>(i)) : 1.0);
}
template <int Q>
__host__ __device__ constexpr int comp(int i, int a) {
  return a == 0 ? cx(i) : (a == 1 ? cy(i) : cz<Q>(i));
}
// Index of the population with velocity +e_a (sign +1) or -e_a (sign -1).
template <int Q>
__host__ __device__ constexpr int axis_pop(int a, int sign) {
  return rest<Q>() + sign * (a == 0 ? 1 : (a == 1 ? 3 : 9));
}
template <int Q>
__host__ __device__ constexpr int nnz(int i) {
  return (cx(i) != 0) + (cy(i) != 0) + (cz<Q>(i) != 0);
}

// ---------------------------------------------------------------------------
// Fast arithmetic.  v_rcp_f32 / v_sqrt_f32 (1 ulp) for the FP32 paths; the FP64
// paths use correctly rounded operations.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return __builtin_sqrt(x); }

// ---------------------------------------------------------------------------
// Storage formats.  Every format stores the deviation d_i = f_i - W_i from the
// rest state.  F16 and BF16 round to nearest even from FP32.
// ---------------------------------------------------------------------------
template <int ST>
struct Store;

template <>
struct Store<LBM_F64> {
  using T = double;
  using R = double;
  static constexpr int bytes = 8;
  __device__ static R dec(T v) { return v; }
  __device__ static T enc(R v) { return v; }
  __device__ static T enc_d(double v) { return v; }
};

template <>
struct Store<LBM_F32> {
  using T = float;
  using R = float;
  static constexpr int bytes = 4;
  __device__ static R dec(T v) { return v; }
  __device__ static T enc(R v) { return v; }
  __device__ static T enc_d(double v) { return (float)v; }
};

template <>
struct Store<LBM_F16_SHIFTED> {
  using T = _Float16;
  using R = float;
  static constexpr int bytes = 2;
  __device__ static R dec(T v) { return (float)v; }
  __device__ static T enc(R v) { return (_Float16)v; }   // v_cvt_f16_f32, nearest even
  __device__ static T enc_d(double v) { return (_Float16)v; }   // one rounding from FP64
};

template <>
struct Store<LBM_BF16_SHIFTED> {
  using T = uint16_t;
  using R = float;
  static constexpr int bytes = 2;
  __device__ static R dec(T v) { return __uint_as_float((uint32_t)v << 16); }
  // Nearest even; one conversion instruction on this target (NaN stays NaN).
  __device__ static T enc(R v) { return __builtin_bit_cast(T, (__bf16)v); }
  // One rounding from FP64: round the binary64 significand to 8 bits
  // (nearest even), after which the conversion to binary32 and the bf16
  // truncation are exact (normal range).
  __device__ static T enc_d(double v) {
    uint64_t b = (uint64_t)__double_as_longlong(v);
    if ((b & 0x7fffffffffffffffull) >= 0x7ff0000000000000ull) return enc((float)v);
    b = (b + 0xfffffffffffull + ((b >> 45) & 1ull)) & ~0x1fffffffffffull;
    return (T)(__float_as_uint((float)__longlong_as_double((long long)b)) >> 16);
  }
};

// ---------------------------------------------------------------------------
// Division by a run-time invariant d >= 1 for n < 2^31 (node indices of an
// instance stay below 2^31).  With l = ceil(log2 d) and M = ceil(2^(31+l)/d),
// which is below 2^32, floor(n/d) = floor(n M / 2^(31+l)): the excess
// M d - 2^(31+l) is below d <= 2^l, so n times it stays below 2^(31+l).  On
// the device that is one 32-bit high multiply and a shift by l - 1.
// ---------------------------------------------------------------------------
struct FastDiv {
  uint32_t M;
  uint32_t shift;
  uint32_t d;
  uint32_t pad;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.pad = 0;
  f.M = 0;
  f.shift = 0;
  if (d >= 2) {
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    f.M = (uint32_t)(((uint64_t(1) << (31 + l)) + d - 1) / d);
    f.shift = l - 1;
  }
  return f;
}

__device__ __forceinline__ uint32_t fdiv_u32(uint32_t n, const FastDiv& f) {
  return f.d <= 1 ? n : __umulhi(n, f.M) >> f.shift;
}

// ---------------------------------------------------------------------------
// Node flags (one byte per node, only for instances with walls, faces other
// than periodic, or a body).
// ---------------------------------------------------------------------------
enum : uint8_t {
  FLAG_SOLID = 1,        // inside the body at the current time
  FLAG_STATIC = 2,       // on a non-periodic face plane (inlet, outlet, wall row)
  FLAG_BODY = 4,         // fluid with a solid lattice neighbour x - c_i
  FLAG_SOLID_NEXT = 8,   // scratch: inside the body at the next time
  FLAG_SPECIAL = FLAG_SOLID | FLAG_STATIC | FLAG_BODY,
};

// Default relative threshold: FP32 paths take gamma from FP64 where
// <Delta|Delta> < kNearEq * (rt^2 + 3 |j|^2), the squared size of the terms
// that cancel in Delta.  FP32 keeps Delta to ~6e-8 of that size, so at the
// threshold gamma is perturbed by ~0.6%, which moves gamma Dh by about the
// FP32 rounding of the populations.  A near-rest node (small rt and j) keeps
// its relative precision and needs no FP64 however small Delta is.
constexpr float kNearEq = 1e-10f;

// Per-instance descriptor read by every kernel (device memory, one per
// instance).  Populations of the instance live at buf + pop_off + i*stride.
struct InstDev {
  int64_t pop_off;
  int64_t stride;
  int64_t N;
  int64_t flag_off;   // byte offset of the instance's flags, -1 if none
  int nx, ny, nz, D;
  FastDiv divx, divy;
  double beta;
  float beta_f;
  float near_eq;      // relative <Delta|Delta> threshold for the FP64 gamma
  int collision;
  int trace_in_s;
  int inlet_profile;
  int ramp_steps;
  int body_kind;
  int face[6];
  double u_in[3];
  double body[16];
  int box_lo[3], box_hi[3];   // swept box of the body
  // Surface mesh (body_kind LBM_BODY_MESH), device arrays of the context:
  // vertices and their velocities (3 doubles each), faces (3 vertex indices
  // each; in 2D segments of the first two).
  const double* mesh_v;
  const double* mesh_vel;
  const int* mesh_f;
  int mesh_nf;
  // Crossings of the lattice lines along x with the surface: the line of
  // column (y, z) = (col_lo[0] + a, col_lo[1] + b), a < col_n[0], b < col_n[1],
  // k = a + col_n[0] b, crosses at x = col_x[col_start[k] .. col_start[k+1]),
  // ascending.  Lines outside the columns do not meet the surface.
  const int* col_start;
  const double* col_x;
  int col_lo[2], col_n[2];
  // Faces by cell of a uniform grid (cell size bin_h from bin_lo, bin_n cells
  // per axis): cell k = a + bin_n[0] (b + bin_n[1] c) lists the faces whose
  // bounding box meets it, bin_face[bin_start[k] .. bin_start[k+1]).
  const int* bin_start;
  const int* bin_face;
  double bin_lo[3];
  double bin_h;
  int bin_n[3];
  // Multiphase forcing (Sec. III.B): on (1) or off, surface-tension and
  // wetting coefficients, and the instance's density, phi and Laplacian
  // fields (N values each; FP64 for FP64 storage, FP32 otherwise), or null
  // when the context steps without the multiphase pipeline.
  int mp;
  double mp_kappa, mp_kappa_w;
  void* mp_field;
};

// A contiguous run of nodes of one instance, processed by one workgroup.
struct Tile {
  int inst;
  int count;
  int64_t node0;
};

// A box region of one instance scanned by the boundary kernel; nodes that lie
// in an earlier region of the same instance are skipped there.
struct Region {
  int inst;
  int first;    // index of the first region of this instance
  int lo[3], hi[3];
};

}  // namespace kbc
