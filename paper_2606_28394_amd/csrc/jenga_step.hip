// Batched block stepping on gfx950: one workgroup (one 64-lane wave) owns a
// "pack" of whole towers for every step of a launch.  Bodies, contact pairs and
// colours stay in LDS; each contact manifold's lever arms, impulses, normal and
// depth live in a per-pack block of device memory, read on every PGS visit with
// the next manifold's record in flight while the current one is solved (this
// keeps LDS per body small, so more waves share a CU).  The step is bound by
// the vector ALUs.  A colour with at most half as many manifolds as threads is
// solved by lane pairs, one body per lane (see pgs_sweeps).  An island too large
// for LDS keeps its layout in device memory, one island per workgroup of eight
// waves (see step_kernel).
//
// Per step (Secs. "Rigid-Body Foundations", "Physics Engine --- Collision
// Detection", "Contact Solver --- Projected Gauss-Seidel (PGS)"):
//   1 external forces: v += dt g + dt F/m (semi-implicit Euler)
//   2 frames: world AABB half sizes, I_w^-1 = R I_b^-1 R^T with R from Eq. (rotmat)
//   3 broadphase (Eq. (aabb)): all same-tower pairs i<j plus the ground, ballot
//     compaction into a small ring that keeps the canonical (i, j) order
//   4 narrowphase: 15-axis SAT on each 64 candidates as soon as the ring holds them
//   5 greedy first-fit colouring over the canonical list (bit masks per body)
//   6 manifolds, written straight into colour-sorted slots: the silhouettes of
//     both boxes along n are zonogons (three projected half-edges); the clipped
//     polygon's extremes along the four diagonals are found among (a) corners of
//     one silhouette inside the other and (b) silhouette edge crossings; points
//     are lifted to the mid-plane of the overlap slab
//   7 PGS: colour by colour, one lane per manifold, its points and rows in
//     order (Eq. (lambda_n) then Eq. (coulomb_pgs) on t1, t2); manifolds of one
//     colour share no dynamic body, so each colour is an exact Gauss-Seidel sweep
//   8 residual of the solve (natural map), reduced per tower over its contiguous
//     canonical range
//   9 integration: x += dt v, q from Eq. (quat_int) with world-frame omega,
//     omega re-derived from the angular momentum (Eq. (newton_euler), torque free)
//  10 Baumgarte correction (Eq. (baumgarte)), colour by colour
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <math.h>
#include <stdint.h>

#include "jenga_device.h"
#include "mlp_device.h"

namespace jg {
namespace {

constexpr uint32_t kGround = 0xffffu;
constexpr int kIslandWaves = 8;   // waves of a workgroup that steps an island in device memory
constexpr int kLatencyWaves = 4;  // waves of a workgroup that steps one tower of a small batch
constexpr int kMaxDevices = 64;

// A barrier among the lanes of one wave.  Every phase runs on one wave (the workgroup's first),
// so this is all its steps need: LDS and device-memory accesses of one wave are performed in
// order.  Only the PGS sweeps of an island in device memory use the whole workgroup and its
// barrier (__syncthreads).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr int kWindows = 4;      // broadphase register windows: packs of up to 256 bodies
constexpr uint32_t kErrCand = 1u, kErrMan = 2u, kErrCol = 4u, kErrNan = 8u;

struct Lds {
  // bodies [comp * nbp + i]
  float *x, *q, *v, *w, *he, *invm, *Iw;
  float* hm;          // AABB half sizes during the broadphase, then colour masks (2 words)
  uint32_t* flag;
  int32_t* tw;
  // towers
  int32_t *tb0, *tb1;
  float* mu;
  uint32_t* tcnt;     // [t*4 + k]: candidates, manifolds, points (launch totals), colours (last step)
  float* tres;        // [t*2 + k]
  int32_t *tc0, *tc1, *tpts;   // canonical range and points of the current step
  uint32_t* tfz;      // [t]: 1 = the tower's state was non-finite at a step's start (held)
  // pushes
  int32_t *pb, *ps, *pn;
  float *pf, *pwd, *px0;
  // colours and scalars
  int32_t *coloff, *colcnt, *scal;
  uint32_t* ring;
  unsigned long long* cyc;   // per-phase cycle counters of this pack
  // canonical colliding pairs (code, colour-sorted position); residual partials afterwards
  uint32_t* cab;
  int32_t* cpos;
  // colour-sorted manifolds
  uint32_t *mab, *mmeta;
  uint32_t *lmlo, *lmhi;   // colouring: per-body lane masks of the current chunk (low, high lanes)
  float* mtb;         // device block after the records: restitution targets, 4 per sorted manifold
  float* md;          // device block, kManDevWords per sorted manifold: r_A [12] (contact frame
                      // (n, t1, t2)), lambda [12], n [3], depth (see mdev)
  float* msat;        // device block after the targets: the narrowphase's normal [3] and depth of
                      // canonical colliding pair p at [4 p]
  // warm start: sorted -> canonical, previous step store (canonical order)
  int32_t* mcanon;
  uint32_t *pkey, *pslot;
  float *pnrm, *plam;
  // learned warm start: network input rows, pre-solve velocities, residual partials,
  // per-tower fallback flag and counters (fallbacks, fallback points)
  uint32_t* xs;
  float *vsave, *rpart;
  uint32_t *tfb, *tfc;
  float* wbox;        // global packs: per 64-body window, AABB lo[3], hi[3] (broadphase)
  uint32_t* cand;     // global packs: the broadphase candidates of a step, canonical order
  uint32_t* cslot;    // global packs: kCandPerBody candidate slots per body (the walk's output)
  int nbp, pc;
};

// the device-block record of sorted manifold m (16-byte aligned: kManDevWords is a multiple of 4)
__device__ __forceinline__ float* mdev(const Lds& L, int m) { return L.md + (size_t)m * kManDevWords; }

// LDS layout mode of a launch (see lds_words)
__device__ __forceinline__ int lds_mode(const StepArgs& a) {
  return a.warm_start == 2 ? 2 : ((a.warm_start == 1 || a.feat_out) ? 1 : 0);
}

// base: the layout (LDS, or device memory for a pack kept there); dev: the pack's block of
// lever arms and impulses in device memory; with use_hot (packs kept in device memory), hot is
// LDS for the small arrays listed in hot_words, and with hot_bodies for the walks' body arrays.
// The flags are compile-time constants at the call, so every array has one address space.
__device__ __forceinline__ Lds carve(float* base, float* dev, float* hot, bool use_hot, bool hot_bodies,
                                     const StepArgs& a) {
  Lds L;
  L.nbp = a.nbp;
  L.pc = a.pc;
  float* p = base;
  auto take = [&](int n) { float* r = p; p += n; return r; };
  const int nb = a.nbp, pc = a.pc, nt = a.tpc, np = a.ppc;
  const int mode = lds_mode(a);
  L.cyc = (unsigned long long*)take(2 * kPhases);   // first: 8-byte aligned
  L.xs = mode == 2 ? (uint32_t*)take(kStageWords) : nullptr;   // 16-byte aligned (80-byte offset)
  // an island's other waves stage their network rows right after the first wave's
  if (use_hot && mode == 2) take((kLearnedIslandWaves - 1) * kStageWords);
  L.x = take(3 * nb); L.q = take(4 * nb); L.v = take(3 * nb); L.w = take(3 * nb);
  L.he = take(3 * nb); L.invm = take(nb);
  L.flag = (uint32_t*)take(nb); L.tw = (int32_t*)take(nb);
  L.Iw = take(6 * nb); L.hm = take(3 * nb);
  L.tb0 = (int32_t*)take(nt); L.tb1 = (int32_t*)take(nt); L.mu = take(nt);
  L.tcnt = (uint32_t*)take(4 * nt); L.tres = take(2 * nt);
  L.tc0 = (int32_t*)take(nt); L.tc1 = (int32_t*)take(nt); L.tpts = (int32_t*)take(nt);
  L.tfz = (uint32_t*)take(nt);
  L.pb = (int32_t*)take(np); L.ps = (int32_t*)take(np); L.pn = (int32_t*)take(np);
  L.pf = take(3 * np); L.pwd = take(np); L.px0 = take(3 * np);
  L.coloff = (int32_t*)take(kMaxColours + 1); L.colcnt = (int32_t*)take(kMaxColours + 1);
  L.scal = (int32_t*)take(16);
  L.ring = (uint32_t*)take(kRing);
  L.cab = (uint32_t*)take(pc); L.cpos = (int32_t*)take(pc);
  L.mab = (uint32_t*)take(pc); L.mmeta = (uint32_t*)take(pc);
  L.md = dev;
  L.mtb = dev + (size_t)kManDevWords * pc;
  L.msat = dev + (size_t)(kManDevWords + kManBiasWords) * pc;
  if (mode >= 1) {
    L.mcanon = (int32_t*)take(pc);
    L.pkey = (uint32_t*)take(pc); L.pslot = (uint32_t*)take(pc); L.pnrm = take(3 * pc); L.plam = take(12 * pc);
  } else {
    L.mcanon = nullptr;
    L.pkey = L.pslot = nullptr;
    L.pnrm = L.plam = nullptr;
  }
  if (mode == 2) {
    L.vsave = take(6 * nb); L.rpart = take(2 * pc);
    L.tfb = (uint32_t*)take(nt); L.tfc = (uint32_t*)take(2 * nt);
  } else {
    L.vsave = L.rpart = nullptr;
    L.tfb = L.tfc = nullptr;
  }
  L.wbox = a.in_gmem ? take((int)window_words(nb)) : nullptr;
  L.cand = a.in_gmem ? (uint32_t*)take(kCandPerBody * nb) : nullptr;
  L.cslot = a.in_gmem ? (uint32_t*)take(kCandPerBody * nb) : nullptr;
  // the colouring's lane masks reuse the sorted-manifold words (free until the manifolds are
  // written)
  L.lmlo = L.mab;
  L.lmhi = L.mmeta;
  if (use_hot) {
    // a pack in device memory keeps its small arrays, and if they fit the arrays its serial
    // walks read, in LDS (the copies in its region stay unused)
    float* h = hot;
    auto htake = [&](int n) { float* r = h; h += n; return r; };
    L.cyc = (unsigned long long*)htake(2 * kPhases);   // first: 8-byte aligned
    L.coloff = (int32_t*)htake(kMaxColours + 1); L.colcnt = (int32_t*)htake(kMaxColours + 1);
    L.scal = (int32_t*)htake(16);
    L.ring = (uint32_t*)htake(kRing);
    L.tb0 = (int32_t*)htake(nt); L.tb1 = (int32_t*)htake(nt); L.mu = htake(nt);
    L.tcnt = (uint32_t*)htake(4 * nt); L.tres = htake(2 * nt);
    L.tc0 = (int32_t*)htake(nt); L.tc1 = (int32_t*)htake(nt); L.tpts = (int32_t*)htake(nt);
    L.tfz = (uint32_t*)htake(nt);
    L.pb = (int32_t*)htake(np); L.ps = (int32_t*)htake(np); L.pn = (int32_t*)htake(np);
    L.pf = htake(3 * np); L.pwd = htake(np); L.px0 = htake(3 * np);
    L.wbox = htake((int)window_words(nb));
    if (hot_bodies) {
      L.x = htake(3 * nb); L.hm = htake(3 * nb); L.flag = (uint32_t*)htake(nb);
      L.lmlo = (uint32_t*)htake(nb); L.lmhi = (uint32_t*)htake(nb);
    }
  }
  return L;
}

__device__ __forceinline__ float dot3(const float a[3], const float b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__device__ __forceinline__ void cross3(const float a[3], const float b[3], float c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
// symmetric 3x3 (xx, yy, zz, xy, xz, yz) times vector
__device__ __forceinline__ void sym_mul(const float I[6], const float c[3], float o[3]) {
  o[0] = I[0] * c[0] + I[3] * c[1] + I[4] * c[2];
  o[1] = I[3] * c[0] + I[1] * c[1] + I[5] * c[2];
  o[2] = I[4] * c[0] + I[5] * c[1] + I[2] * c[2];
}

// Eq. (rotmat), row-major
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float R[9]) {
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - z * w);       R[2] = 2.f * (x * z + y * w);
  R[3] = 2.f * (x * y + z * w);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - x * w);
  R[6] = 2.f * (x * z - y * w);       R[7] = 2.f * (y * z + x * w);       R[8] = 1.f - 2.f * (x * x + y * y);
}

__device__ __forceinline__ void body_R(const Lds& L, int i, float R[9]) {
  const int nb = L.nbp;
  quat_rot(L.q[i], L.q[nb + i], L.q[2 * nb + i], L.q[3 * nb + i], R);
}
__device__ __forceinline__ void load3(const float* a, int stride, int i, float o[3]) {
  o[0] = a[i]; o[1] = a[stride + i]; o[2] = a[2 * stride + i];
}
__device__ __forceinline__ void store3(float* a, int stride, int i, const float o[3]) {
  a[i] = o[0]; a[stride + i] = o[1]; a[2 * stride + i] = o[2];
}

// The contact-frame arithmetic below (basis, rotations into and out of the frame) is written
// with explicit fused multiply-adds and no other contraction: a PGS visit then gives the same
// bits whether one lane works both bodies or a lane pair works one body each, whatever the
// compiler would fuse in either code.
__device__ __forceinline__ float dot3x(const float a[3], const float b[3]) {
#pragma clang fp contract(off)
  return __builtin_fmaf(a[0], b[0], __builtin_fmaf(a[1], b[1], a[2] * b[2]));
}
__device__ __forceinline__ void sym_mulx(const float I[6], const float c[3], float o[3]) {
#pragma clang fp contract(off)
  o[0] = __builtin_fmaf(I[0], c[0], __builtin_fmaf(I[3], c[1], I[4] * c[2]));
  o[1] = __builtin_fmaf(I[3], c[0], __builtin_fmaf(I[1], c[1], I[5] * c[2]));
  o[2] = __builtin_fmaf(I[4], c[0], __builtin_fmaf(I[5], c[1], I[2] * c[2]));
}

__device__ __forceinline__ void tangent_basis(const float n[3], float t1[3], float t2[3]) {
#pragma clang fp contract(off)
  float e[3] = {0.f, 0.f, 0.f};
  if (fabsf(n[0]) < 0.9f) e[0] = 1.f; else e[1] = 1.f;
  const float en = dot3x(e, n);
  float t[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = __builtin_fmaf(-en, n[k], e[k]);
  const float il = __builtin_amdgcn_rsqf(dot3x(t, t));   // |t|^2 >= 0.19: no denormal scaling
  t1[0] = t[0] * il; t1[1] = t[1] * il; t1[2] = t[2] * il;
  t2[0] = __builtin_fmaf(n[1], t1[2], -(n[2] * t1[1]));
  t2[1] = __builtin_fmaf(n[2], t1[0], -(n[0] * t1[2]));
  t2[2] = __builtin_fmaf(n[0], t1[1], -(n[1] * t1[0]));
}

// ------------------------------------------------------------------------------------------------
// narrowphase: 15-axis SAT in coordinates relative to A's centre (d = xB - xA)
// ------------------------------------------------------------------------------------------------
// kPreferFace (reference-face manifolds): of a colliding pair, the normal and depth come from the
// best face axis unless the best cross axis is smaller than 0.95 of it by more than 1 um, so that
// a cross axis parallel to a face normal (crossed blocks: x_A x y_B = z) never stands in for it
template <bool kPreferFace = false>
__device__ __forceinline__ bool sat_boxes(const float RA[9], const float heA[3], const float RB[9], const float heB[3],
                          const float d[3], float n[3], float& depth, int* axis_out = nullptr) {
  float A[3][3], B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) { A[i][k] = RA[3 * k + i]; B[i][k] = RB[3 * k + i]; }
  float best = INFINITY;
  float bu[3] = {0.f, 0.f, 1.f};
  int bi = 0;
  bool sep = false;
  auto axis = [&](const float u[3], int idx) {
    const float ra = heA[0] * fabsf(dot3(A[0], u)) + heA[1] * fabsf(dot3(A[1], u)) + heA[2] * fabsf(dot3(A[2], u));
    const float rb = heB[0] * fabsf(dot3(B[0], u)) + heB[1] * fabsf(dot3(B[1], u)) + heB[2] * fabsf(dot3(B[2], u));
    const float dd = ra + rb - fabsf(dot3(d, u));
    sep = sep || !(dd > 0.f);
    if (dd < best) { best = dd; bu[0] = u[0]; bu[1] = u[1]; bu[2] = u[2]; bi = idx; }
  };
#pragma unroll
  for (int i = 0; i < 3; ++i) axis(A[i], i);
#pragma unroll
  for (int j = 0; j < 3; ++j) axis(B[j], 3 + j);
  if (sep) return false;
  const float best_face = best;
  const float bu_face[3] = {bu[0], bu[1], bu[2]};
  const int bi_face = bi;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float c[3];
      cross3(A[i], B[j], c);
      const float len2 = dot3(c, c);
      if (len2 < 1e-10f) continue;          // |a x b| < 1e-5: not tested
      const float il = rsqrtf(len2);
      c[0] *= il; c[1] *= il; c[2] *= il;
      axis(c, 6 + 3 * i + j);
    }
  if (sep) return false;
  if (kPreferFace && bi >= 6 && !(best < 0.95f * best_face - 1e-6f)) {
    best = best_face;
    bu[0] = bu_face[0]; bu[1] = bu_face[1]; bu[2] = bu_face[2];
    bi = bi_face;
  }
  const float s = dot3(d, bu) < 0.f ? -1.f : 1.f;
  n[0] = s * bu[0]; n[1] = s * bu[1]; n[2] = s * bu[2];
  depth = best;
  if (axis_out) *axis_out = bi;
  return true;
}

// ------------------------------------------------------------------------------------------------
// manifold of a colliding box pair (relative to A's centre)
// ------------------------------------------------------------------------------------------------
struct V2 { float x, y; };
__device__ __forceinline__ float cr2(V2 a, V2 b) { return a.x * b.y - a.y * b.x; }

struct Zono {        // silhouette of a box along n: centre + sum_i s_i g_i, |s_i| <= 1
  V2 c, g[3];
  V2 m[3];           // slab normals perp(g_i)
  float h[3];        // slab half widths
  float tol[3];
  bool use[3];
};

__device__ __forceinline__ void zono_build(Zono& Z) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Z.m[k].x = -Z.g[k].y; Z.m[k].y = Z.g[k].x;
    float hk = 0.f;
#pragma unroll
    for (int j = 0; j < 3; ++j) hk += fabsf(Z.m[k].x * Z.g[j].x + Z.m[k].y * Z.g[j].y);
    Z.h[k] = hk;
    const float len = sqrtf(Z.g[k].x * Z.g[k].x + Z.g[k].y * Z.g[k].y);
    Z.use[k] = len > 1e-9f;
    Z.tol[k] = 2e-7f * len;
  }
}

__device__ __forceinline__ bool zono_inside(const Zono& Z, V2 p) {
  const float px = p.x - Z.c.x, py = p.y - Z.c.y;
  bool in = true;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    in = in && (!Z.use[k] || fabsf(Z.m[k].x * px + Z.m[k].y * py) <= Z.h[k] + Z.tol[k]);
  return in;
}

// CCW hexagon (possibly with repeated or collinear vertices) of the zonogon
__device__ __forceinline__ void zono_hexagon(const Zono& Z, V2 v[6]) {
  V2 g[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g[k] = Z.g[k];
    if (g[k].y < 0.f || (g[k].y == 0.f && g[k].x < 0.f)) { g[k].x = -g[k].x; g[k].y = -g[k].y; }
  }
  // sort by polar angle in [0, pi): a before b when cross(a, b) > 0
  auto cswap = [](V2& a, V2& b) { if (cr2(a, b) < 0.f) { V2 t = a; a = b; b = t; } };
  cswap(g[0], g[1]); cswap(g[1], g[2]); cswap(g[0], g[1]);
  v[0].x = Z.c.x - (g[0].x + g[1].x + g[2].x); v[0].y = Z.c.y - (g[0].y + g[1].y + g[2].y);
  v[1].x = v[0].x + 2.f * g[0].x; v[1].y = v[0].y + 2.f * g[0].y;
  v[2].x = v[1].x + 2.f * g[1].x; v[2].y = v[1].y + 2.f * g[1].y;
  v[3].x = v[2].x + 2.f * g[2].x; v[3].y = v[2].y + 2.f * g[2].y;
  v[4].x = v[3].x - 2.f * g[0].x; v[4].y = v[3].y - 2.f * g[0].y;
  v[5].x = v[4].x - 2.f * g[1].x; v[5].y = v[4].y - 2.f * g[1].y;
}

struct Extremes {
  float best[4];
  V2 p[4];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int s = 0; s < 4; ++s) { best[s] = -INFINITY; p[s].x = p[s].y = 0.f; }
  }
  // diagonals (+,+), (-,+), (-,-), (+,-); the first candidate wins ties
  __device__ __forceinline__ void consider(V2 q) {
    const float a = q.x + q.y, b = q.y - q.x;
    if (a > best[0]) { best[0] = a; p[0] = q; }
    if (b > best[1]) { best[1] = b; p[1] = q; }
    if (-a > best[2]) { best[2] = -a; p[2] = q; }
    if (-b > best[3]) { best[3] = -b; p[3] = q; }
  }
};

// Points relative to A's centre, in contact-frame coordinates (along n, t1, t2), in slot
// order; bit s of the result marks slot s as used.
__device__ __forceinline__ uint32_t manifold_boxes(const float RA[9], const float heA[3], const float RB[9], const float heB[3],
                                   const float d[3], const float n[3], float t1[3], float rA[4][3]) {
  float t2[3];
  tangent_basis(n, t1, t2);
  Zono ZA, ZB;
  float zA = 0.f, zB = dot3(d, n);
  ZA.c.x = 0.f; ZA.c.y = 0.f;
  ZB.c.x = dot3(d, t1); ZB.c.y = dot3(d, t2);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float a[3] = {RA[i], RA[3 + i], RA[6 + i]};
    const float b[3] = {RB[i], RB[3 + i], RB[6 + i]};
    ZA.g[i].x = heA[i] * dot3(a, t1); ZA.g[i].y = heA[i] * dot3(a, t2);
    ZB.g[i].x = heB[i] * dot3(b, t1); ZB.g[i].y = heB[i] * dot3(b, t2);
    zA += heA[i] * fabsf(dot3(a, n));
    zB -= heB[i] * fabsf(dot3(b, n));
  }
  zono_build(ZA);
  zono_build(ZB);
  Extremes E;
  E.init();
  bool any = false;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float s0 = (k & 1) ? 1.f : -1.f, s1 = (k & 2) ? 1.f : -1.f, s2 = (k & 4) ? 1.f : -1.f;
    V2 pa, pb;
    pa.x = s0 * ZA.g[0].x + s1 * ZA.g[1].x + s2 * ZA.g[2].x;
    pa.y = s0 * ZA.g[0].y + s1 * ZA.g[1].y + s2 * ZA.g[2].y;
    pb.x = ZB.c.x + s0 * ZB.g[0].x + s1 * ZB.g[1].x + s2 * ZB.g[2].x;
    pb.y = ZB.c.y + s0 * ZB.g[0].y + s1 * ZB.g[1].y + s2 * ZB.g[2].y;
    if (zono_inside(ZB, pa)) { E.consider(pa); any = true; }
    if (zono_inside(ZA, pb)) { E.consider(pb); any = true; }
  }
  V2 ha[6], hb[6];
  zono_hexagon(ZA, ha);
  zono_hexagon(ZB, hb);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const V2 p0 = ha[i], p1 = ha[(i + 1) % 6];
    const V2 u = {p1.x - p0.x, p1.y - p0.y};
    const float lu = u.x * u.x + u.y * u.y;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const V2 q0 = hb[j], q1 = hb[(j + 1) % 6];
      const V2 w = {q1.x - q0.x, q1.y - q0.y};
      const float den = cr2(u, w);
      const float lw = w.x * w.x + w.y * w.y;
      if (lu < 1e-18f || den * den <= 1e-12f * lu * lw) continue;   // empty or parallel edges
      const V2 r = {q0.x - p0.x, q0.y - p0.y};
      const float id = 1.f / den;
      const float t = cr2(r, w) * id, s = cr2(r, u) * id;
      if (t >= -1e-6f && t <= 1.f + 1e-6f && s >= -1e-6f && s <= 1.f + 1e-6f) {
        V2 pt = {p0.x + t * u.x, p0.y + t * u.y};
        E.consider(pt);
        any = true;
      }
    }
  }
  const float zmid = 0.5f * (zA + zB);
  if (!any) {
    // empty clip: halfway between the support corners of A (max along n) and B (min)
    float ba = -INFINITY, bb = INFINITY;
    float ca[3] = {0, 0, 0}, cb[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float s[3] = {(k & 1) ? heA[0] : -heA[0], (k & 2) ? heA[1] : -heA[1], (k & 4) ? heA[2] : -heA[2]};
      const float sb[3] = {(k & 1) ? heB[0] : -heB[0], (k & 2) ? heB[1] : -heB[1], (k & 4) ? heB[2] : -heB[2]};
      float pa[3], pb[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        pa[r] = RA[3 * r] * s[0] + RA[3 * r + 1] * s[1] + RA[3 * r + 2] * s[2];
        pb[r] = d[r] + RB[3 * r] * sb[0] + RB[3 * r + 1] * sb[1] + RB[3 * r + 2] * sb[2];
      }
      const float da = dot3(pa, n), db = dot3(pb, n);
      if (da > ba) { ba = da; ca[0] = pa[0]; ca[1] = pa[1]; ca[2] = pa[2]; }
      if (db < bb) { bb = db; cb[0] = pb[0]; cb[1] = pb[1]; cb[2] = pb[2]; }
    }
    float mid[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) mid[r] = 0.5f * (ca[r] + cb[r]);
    rA[0][0] = dot3(mid, n); rA[0][1] = dot3(mid, t1); rA[0][2] = dot3(mid, t2);
    return 1u;
  }
  uint32_t used = 0u;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    bool ok = E.best[s] != -INFINITY;
#pragma unroll
    for (int c = 0; c < s; ++c) {
      const float dx = E.p[s].x - E.p[c].x, dy = E.p[s].y - E.p[c].y;
      ok = ok && !(((used >> c) & 1u) && (dx * dx + dy * dy < 1e-12f));
    }
    if (ok) used |= 1u << s;
    rA[s][0] = zmid; rA[s][1] = E.p[s].x; rA[s][2] = E.p[s].y;
  }
  return used;
}

// Reference-face clipping (the alternative to the literal silhouettes), relative to A's centre in
// the contact frame.  For a face axis, the face that owns it is the reference face and the other
// box's face most opposed to it the incident face; both are parallelograms in the (t1, t2) plane
// (projections along n, which is the reference face's normal).  The clipped polygon's vertices
// are incident corners inside the reference rectangle, reference corners inside the incident
// parallelogram and crossings of their edges; each carries the incident face's height along n
// there, and those on or below the reference face are kept, lifted halfway to it.  The slots are
// the kept vertices extreme along the four diagonals.  An edge axis gives one point, the midpoint
// of the closest points of the two supporting edges.  Returns the used-slot bits (0: nothing on or
// below the reference face; the caller then takes the silhouettes' manifold).
struct ExtremesZ {
  float best[4];
  V2 p[4];
  float z[4];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int s = 0; s < 4; ++s) { best[s] = -INFINITY; p[s].x = p[s].y = 0.f; z[s] = 0.f; }
  }
  __device__ __forceinline__ void consider(V2 q, float zq) {
    const float a = q.x + q.y, b = q.y - q.x;
    if (a > best[0]) { best[0] = a; p[0] = q; z[0] = zq; }
    if (b > best[1]) { best[1] = b; p[1] = q; z[1] = zq; }
    if (-a > best[2]) { best[2] = -a; p[2] = q; z[2] = zq; }
    if (-b > best[3]) { best[3] = -b; p[3] = q; z[3] = zq; }
  }
};

__device__ __forceinline__ uint32_t manifold_refface(const float RA[9], const float heA[3], const float RB[9],
                                                     const float heB[3], const float d[3], const float n[3], int axis,
                                                     float t1[3], float rA[4][3]) {
  float t2[3];
  tangent_basis(n, t1, t2);
  float A[3][3], B[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) { A[i][k] = RA[3 * k + i]; B[i][k] = RB[3 * k + i]; }
  if (axis >= 6) {
    const int i = (axis - 6) / 3, j = (axis - 6) % 3;
    float pa[3] = {0.f, 0.f, 0.f}, pb[3] = {d[0], d[1], d[2]};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (q != i) {
        const float sg = dot3(n, A[q]) >= 0.f ? heA[q] : -heA[q];
#pragma unroll
        for (int k = 0; k < 3; ++k) pa[k] += sg * A[q][k];
      }
      if (q != j) {
        const float sg = dot3(n, B[q]) >= 0.f ? -heB[q] : heB[q];
#pragma unroll
        for (int k = 0; k < 3; ++k) pb[k] += sg * B[q][k];
      }
    }
    float r[3], c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = pa[k] - pb[k];
    cross3(A[i], B[j], c);
    const float det = dot3(c, c), a12 = dot3(A[i], B[j]);
    const float ar = dot3(A[i], r), br = dot3(B[j], r);
    float sa = det > 1e-12f ? (a12 * br - ar) / det : 0.f;
    sa = fminf(fmaxf(sa, -heA[i]), heA[i]);
    float tb = fminf(fmaxf(br + a12 * sa, -heB[j]), heB[j]);
    sa = fminf(fmaxf(a12 * tb - ar, -heA[i]), heA[i]);
    float mid[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) mid[k] = 0.5f * ((pa[k] + sa * A[i][k]) + (pb[k] + tb * B[j][k]));
    rA[0][0] = dot3(mid, n); rA[0][1] = dot3(mid, t1); rA[0][2] = dot3(mid, t2);
    return 1u;
  }
  const bool refA = axis < 3;
  const int fi = refA ? axis : axis - 3;
  const int s1 = fi == 0 ? 1 : 0, s2 = fi == 2 ? 1 : 2;
  const float un = refA ? 1.f : -1.f;           // u = un n, from the reference box to the other
  // reference face: centre (relative to A) and its two half edges, projected
  float cr[3], fr[3], e1r[3], e2r[3];
  float hr1, hr2, hrf;
  if (refA) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { fr[k] = A[fi][k]; e1r[k] = A[s1][k]; e2r[k] = A[s2][k]; }
    hrf = heA[fi]; hr1 = heA[s1]; hr2 = heA[s2];
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) { fr[k] = B[fi][k]; e1r[k] = B[s1][k]; e2r[k] = B[s2][k]; }
    hrf = heB[fi]; hr1 = heB[s1]; hr2 = heB[s2];
  }
  const float su = un * dot3(n, fr) >= 0.f ? hrf : -hrf;
#pragma unroll
  for (int k = 0; k < 3; ++k) cr[k] = (refA ? 0.f : d[k]) + su * fr[k];
  const float zr = dot3(cr, n);                 // the reference face's height along n
  const V2 crc = {dot3(cr, t1), dot3(cr, t2)};
  const V2 g1 = {hr1 * dot3(e1r, t1), hr1 * dot3(e1r, t2)}, g2 = {hr2 * dot3(e2r, t1), hr2 * dot3(e2r, t2)};
  // incident face: the other box's face most opposed to u
  float I[3][3], heI[3], xi[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int k = 0; k < 3; ++k) I[q][k] = refA ? B[q][k] : A[q][k];
    heI[q] = refA ? heB[q] : heA[q];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) xi[k] = refA ? d[k] : 0.f;
  int fk = 0;
  float bestd = -1.f;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float dq = fabsf(dot3(n, I[q]));
    if (dq > bestd) { bestd = dq; fk = q; }
  }
  const int k1 = fk == 0 ? 1 : 0, k2 = fk == 2 ? 1 : 2;
  float fI[3], a1[3], a2[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { fI[k] = I[fk][k]; a1[k] = I[k1][k]; a2[k] = I[k2][k]; }
  const float sf = un * dot3(n, fI) >= 0.f ? -heI[fk] : heI[fk];
  float ci[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) ci[k] = xi[k] + sf * fI[k];
  const V2 cic = {dot3(ci, t1), dot3(ci, t2)};
  const float zc = dot3(ci, n);
  const V2 h1 = {heI[k1] * dot3(a1, t1), heI[k1] * dot3(a1, t2)}, h2 = {heI[k2] * dot3(a2, t1), heI[k2] * dot3(a2, t2)};
  const float dz1 = heI[k1] * dot3(a1, n), dz2 = heI[k2] * dot3(a2, n);
  // on or below the reference face: u . (p - cr) <= 0, i.e. un (z - zr) <= 0
  ExtremesZ E;
  E.init();
  bool any = false;
  auto keep = [&](V2 q, float z) {
    if (un * (z - zr) <= 0.f) {
      E.consider(q, 0.5f * (z + zr));
      any = true;
    }
  };
  const float gg1 = g1.x * g1.x + g1.y * g1.y, gg2 = g2.x * g2.x + g2.y * g2.y;
  const float deth = cr2(h1, h2);
  V2 ic[4], rc[4];
  float iz[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float sa = (c == 0 || c == 3) ? 1.f : -1.f, sb = (c < 2) ? 1.f : -1.f;
    ic[c].x = cic.x + sa * h1.x + sb * h2.x;
    ic[c].y = cic.y + sa * h1.y + sb * h2.y;
    iz[c] = zc + sa * dz1 + sb * dz2;
    rc[c].x = crc.x + sa * g1.x + sb * g2.x;
    rc[c].y = crc.y + sa * g1.y + sb * g2.y;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    // incident corner inside the reference rectangle (orthogonal half edges)
    const float px = ic[c].x - crc.x, py = ic[c].y - crc.y;
    const float a = (px * g1.x + py * g1.y) / gg1, b = (px * g2.x + py * g2.y) / gg2;
    if (fabsf(a) <= 1.f + 1e-6f && fabsf(b) <= 1.f + 1e-6f) keep(ic[c], iz[c]);
    // reference corner inside the incident parallelogram, at the incident face's height there
    const V2 rq = {rc[c].x - cic.x, rc[c].y - cic.y};
    const float ai = cr2(rq, h2) / deth, bi = cr2(h1, rq) / deth;
    if (fabsf(ai) <= 1.f + 1e-6f && fabsf(bi) <= 1.f + 1e-6f) keep(rc[c], zc + ai * dz1 + bi * dz2);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const V2 p0 = ic[c], p1 = ic[(c + 1) & 3];
    const V2 u = {p1.x - p0.x, p1.y - p0.y};
    const float lu = u.x * u.x + u.y * u.y;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const V2 q0 = rc[e], q1 = rc[(e + 1) & 3];
      const V2 w = {q1.x - q0.x, q1.y - q0.y};
      const float den = cr2(u, w);
      const float lw = w.x * w.x + w.y * w.y;
      if (lu < 1e-18f || den * den <= 1e-12f * lu * lw) continue;
      const V2 r = {q0.x - p0.x, q0.y - p0.y};
      const float idn = 1.f / den;
      const float t = cr2(r, w) * idn, sv = cr2(r, u) * idn;
      if (t >= -1e-6f && t <= 1.f + 1e-6f && sv >= -1e-6f && sv <= 1.f + 1e-6f) {
        const V2 pt = {p0.x + t * u.x, p0.y + t * u.y};
        keep(pt, iz[c] + t * (iz[(c + 1) & 3] - iz[c]));
      }
    }
  }
  if (!any) return 0u;
  uint32_t used = 0u;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    bool ok = E.best[s] != -INFINITY;
#pragma unroll
    for (int c = 0; c < s; ++c) {
      const float dx = E.p[s].x - E.p[c].x, dy = E.p[s].y - E.p[c].y;
      ok = ok && !(((used >> c) & 1u) && (dx * dx + dy * dy < 1e-12f));
    }
    if (ok) used |= 1u << s;
    rA[s][0] = E.z[s]; rA[s][1] = E.p[s].x; rA[s][2] = E.p[s].y;
  }
  return used;
}

// ------------------------------------------------------------------------------------------------
// PGS rows (Eq. (lambda_n), Eq. (coulomb_pgs)), worked in the contact frame F = (n, t1, t2).
// In that frame a row's direction is a unit axis e_K, so r x e_K has two non-zero components
// and an impulse changes one linear-velocity component; A gets -P, B gets +P.
// ------------------------------------------------------------------------------------------------
struct Frame { float f[3][3]; };   // rows n, t1, t2 (right handed: t2 = n x t1)

__device__ __forceinline__ void make_frame(const float n[3], Frame& F) {
  F.f[0][0] = n[0]; F.f[0][1] = n[1]; F.f[0][2] = n[2];
  tangent_basis(n, F.f[1], F.f[2]);
}
__device__ __forceinline__ void to_local(const Frame& F, const float v[3], float o[3]) {
  o[0] = dot3x(F.f[0], v); o[1] = dot3x(F.f[1], v); o[2] = dot3x(F.f[2], v);
}
__device__ __forceinline__ void to_world(const Frame& F, const float o[3], float v[3]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int r = 0; r < 3; ++r) v[r] = __builtin_fmaf(F.f[0][r], o[0], __builtin_fmaf(F.f[1][r], o[1], F.f[2][r] * o[2]));
}

// body velocities and inverse inertia in the contact frame.  v0, w0 keep the velocities as
// loaded: only the change is rotated back, so the frame's rounding (F^T F = I + O(eps)) touches
// the impulses' effect and not the whole velocity on every visit.
struct LBody {
  float v[3], w[3], v0[3], w0[3], I[6], im;   // I: (00, 11, 22, 01, 02, 12)
  bool dyn;
};

__device__ constexpr int sym_index(int r, int c) {
  return r == c ? r : ((r + c == 1) ? 3 : ((r + c == 2) ? 4 : 5));
}

// A body without mass holds zero velocity, inverse mass and inverse inertia in the pack (its
// stored velocity is left as given), so it needs no case of its own; the ground (i = kGround,
// only ever the second body of a pair) reads slot 0 and takes zeros.
__device__ __forceinline__ void load_local_g(const Lds& L, int i, bool ground, const Frame& F, LBody& b) {
  const int nb = L.nbp;
  const int j = ground ? 0 : i;
  float v[3], w[3], Iw[6];
  load3(L.v, nb, j, v);
  load3(L.w, nb, j, w);
#pragma unroll
  for (int k = 0; k < 6; ++k) Iw[k] = L.Iw[k * nb + j];
  float im = L.invm[j];
  if (ground) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { v[k] = 0.f; w[k] = 0.f; }
#pragma unroll
    for (int k = 0; k < 6; ++k) Iw[k] = 0.f;
    im = 0.f;
  }
  to_local(F, v, b.v);
  to_local(F, w, b.w);
#pragma unroll
  for (int k = 0; k < 3; ++k) { b.v0[k] = b.v[k]; b.w0[k] = b.w[k]; }
  // F Iw F^T
  float g[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) sym_mulx(Iw, F.f[j], g[j]);
  b.I[0] = dot3x(F.f[0], g[0]); b.I[1] = dot3x(F.f[1], g[1]); b.I[2] = dot3x(F.f[2], g[2]);
  b.I[3] = dot3x(F.f[0], g[1]); b.I[4] = dot3x(F.f[0], g[2]); b.I[5] = dot3x(F.f[1], g[2]);
  b.im = im;
  b.dyn = im > 0.f;
}
template <bool kMayBeGround>
__device__ __forceinline__ void load_local(const Lds& L, int i, const Frame& F, LBody& b) {
  load_local_g(L, i, kMayBeGround && i == (int)kGround, F, b);
}

__device__ __forceinline__ void store_local(const Lds& L, int i, const Frame& F, const LBody& b) {
  if (!b.dyn) return;
  float dv[3], dw[3], v[3], w[3], gv[3], gw[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { dv[k] = b.v[k] - b.v0[k]; dw[k] = b.w[k] - b.w0[k]; }
  to_world(F, dv, gv);
  to_world(F, dw, gw);
  load3(L.v, L.nbp, i, v);
  load3(L.w, L.nbp, i, w);
#pragma unroll
  for (int k = 0; k < 3; ++k) { v[k] += gv[k]; w[k] += gw[k]; }
  store3(L.v, L.nbp, i, v);
  store3(L.w, L.nbp, i, w);
}

// The inverse body-frame inertia of box i of mass m (as given), Eq. (inertia) with l, w, h the
// full sizes (2 h_k): 1 / (m (w^2 + h^2) / 12) about the length axis and likewise about the
// others; zero for a body without mass.  Taken where it is needed (the mass from device memory),
// so the pack holds no copy of it.
__device__ __forceinline__ void inv_body_inertia(const Lds& L, int i, float m, float o[3]) {
  const int NB = L.nbp;
  const float l = 2.f * L.he[i], wd = 2.f * L.he[NB + i], hh = 2.f * L.he[2 * NB + i];
  const bool dyn = m > 0.f;
  o[0] = dyn ? 1.f / (m / 12.f * (wd * wd + hh * hh)) : 0.f;
  o[1] = dyn ? 1.f / (m / 12.f * (l * l + hh * hh)) : 0.f;
  o[2] = dyn ? 1.f / (m / 12.f * (l * l + wd * wd)) : 0.f;
}

// the two non-zero components (at i1 < i2) of a x e_K
template <int K>
__device__ __forceinline__ void axis_cross(const float a[3], float& c1, float& c2) {
  if constexpr (K == 0) { c1 = a[2]; c2 = -a[1]; }        // (0, a2, -a1)
  else if constexpr (K == 1) { c1 = -a[2]; c2 = a[0]; }   // (-a2, 0, a0)
  else { c1 = a[1]; c2 = -a[0]; }                         // (a1, -a0, 0)
}

template <int K>
struct RowTerms {
  static constexpr int i1 = (K == 0) ? 1 : 0;
  static constexpr int i2 = (K == 2) ? 1 : 2;
  float a1, a2, b1, b2;   // r_A x e_K, r_B x e_K
  float iA[3], iB[3];     // I_A^-1 (r_A x e_K), I_B^-1 (r_B x e_K)
  float k;                // inverse effective mass, Eq. (keff)
  __device__ __forceinline__ void build(const LBody& A, const LBody& B, const float rA[3], const float rB[3]) {
    axis_cross<K>(rA, a1, a2);
    axis_cross<K>(rB, b1, b2);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      iA[r] = A.I[sym_index(r, i1)] * a1 + A.I[sym_index(r, i2)] * a2;
      iB[r] = B.I[sym_index(r, i1)] * b1 + B.I[sym_index(r, i2)] * b2;
    }
    k = A.im + B.im + (a1 * iA[i1] + a2 * iA[i2]) + (b1 * iB[i1] + b2 * iB[i2]);
  }
  __device__ __forceinline__ float vrel(const LBody& A, const LBody& B) const {
    return (B.v[K] - A.v[K]) + (b1 * B.w[i1] + b2 * B.w[i2]) - (a1 * A.w[i1] + a2 * A.w[i2]);
  }
  __device__ __forceinline__ void apply(LBody& A, LBody& B, float dl) const {
    A.v[K] -= A.im * dl;
    B.v[K] += B.im * dl;
#pragma unroll
    for (int q = 0; q < 3; ++q) { A.w[q] -= dl * iA[q]; B.w[q] += dl * iB[q]; }
  }
};

__device__ __forceinline__ void manifold_open(const Lds& L, uint32_t ab, const float n[3], int& a, int& b, Frame& F,
                                              LBody& A, LBody& B, float dAB[3]) {
  a = (int)(ab >> 16);
  b = (int)(ab & 0xffffu);
  make_frame(n, F);
  load_local<false>(L, a, F, A);
  load_local<true>(L, b, F, B);
  if (b != (int)kGround) {
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = L.x[k * L.nbp + a] - L.x[k * L.nbp + b];
    to_local(F, d, dAB);
  } else {
    dAB[0] = dAB[1] = dAB[2] = 0.f;
  }
}

__device__ __forceinline__ void manifold_open(const Lds& L, int m, int& a, int& b, Frame& F, LBody& A, LBody& B,
                                              float dAB[3]) {
  const float n[3] = {mdev(L, m)[24], mdev(L, m)[25], mdev(L, m)[26]};
  manifold_open(L, L.mab[m], n, a, b, F, A, B, dAB);
}

__device__ __forceinline__ void load_point(const Lds& L, int m, int j, const float dAB[3], float rA[3], float rB[3],
                                  float lam[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    rA[k] = mdev(L, m)[j * 3 + k];
    rB[k] = rA[k] + dAB[k];
    lam[k] = mdev(L, m)[12 + j * 3 + k];
  }
}

// One body's share of a PGS row, written out with explicit fused multiply-adds and no other
// contraction, so that a row gives the same bits whether one lane works both bodies or two
// lanes work one body each (the partial sums below are then swapped between the lanes).
template <int K>
struct SideRow {
  static constexpr int i1 = (K == 0) ? 1 : 0;
  static constexpr int i2 = (K == 2) ? 1 : 2;
  float c1, c2;   // r x e_K
  float i[3];     // I^-1 (r x e_K)
  __device__ __forceinline__ void build(const LBody& s, const float r[3]) {
#pragma clang fp contract(off)
    axis_cross<K>(r, c1, c2);
#pragma unroll
    for (int q = 0; q < 3; ++q) i[q] = __builtin_fmaf(s.I[sym_index(q, i1)], c1, s.I[sym_index(q, i2)] * c2);
  }
  // the body's term of the inverse effective mass, Eq. (keff)
  __device__ __forceinline__ float kpart(const LBody& s) const {
#pragma clang fp contract(off)
    return __builtin_fmaf(c1, i[i1], __builtin_fmaf(c2, i[i2], s.im));
  }
  // the velocity of the body's contact point along e_K
  __device__ __forceinline__ float vpart(const LBody& s) const {
#pragma clang fp contract(off)
    return __builtin_fmaf(c1, s.w[i1], __builtin_fmaf(c2, s.w[i2], s.v[K]));
  }
  // impulse sdl along e_K on the body (A takes -dl, B takes +dl)
  __device__ __forceinline__ void apply(LBody& s, float sdl) const {
    s.v[K] = __builtin_fmaf(s.im, sdl, s.v[K]);
#pragma unroll
    for (int q = 0; q < 3; ++q) s.w[q] = __builtin_fmaf(sdl, i[q], s.w[q]);
  }
};

// solver options of a launch: restitution e; cone: the tangent pair projected onto the disc of
// radius mu lambda_n instead of each tangent clipped; bias: the normal row drives the point's
// normal velocity to its pre-solve target -e min(0, v_n-) instead of applying (1 + e) to the
// current velocity
struct SolveOpts {
  float e;
  bool cone, bias;
};

// the row's new impulse from its relative velocity u and the reciprocal rk of its inverse
// effective mass k: Eq. (lambda_n) with restitution for the normal row, the clipped
// Eq. (coulomb_pgs) for a tangent
template <bool kNormal>
__device__ __forceinline__ float row_lambda_rk(float lam, float u, float rk, float bound, const SolveOpts& o,
                                               float target) {
#pragma clang fp contract(off)
  if constexpr (kNormal) {
    if (o.bias) return fmaxf(__builtin_fmaf(target - u, rk, lam), 0.f);
    return fmaxf(__builtin_fmaf(-((1.f + o.e) * u), rk, lam), 0.f);
  } else {
    return fminf(fmaxf(__builtin_fmaf(-u, rk, lam), -bound), bound);
  }
}
template <bool kNormal>
__device__ __forceinline__ float row_lambda(float lam, float u, float k, float bound, const SolveOpts& o,
                                            float target) {
  return row_lambda_rk<kNormal>(lam, u, __builtin_amdgcn_rcpf(k), bound, o, target);
}

// the tangent pair's unclipped new impulses projected onto the disc of radius b (both lanes of a
// pair compute it from the same bits)
__device__ __forceinline__ void disc_project(float& l1, float& l2, float b) {
#pragma clang fp contract(off)
  const float s2 = __builtin_fmaf(l1, l1, l2 * l2);
  if (s2 > b * b) {
    const float f = b * __builtin_amdgcn_rsqf(s2);
    l1 *= f;
    l2 *= f;
  }
}

// one row on one lane, both bodies
template <int K>
__device__ __forceinline__ void row_single(LBody& A, LBody& B, const float rA[3], const float rB[3], float& lam,
                                           float bound, const SolveOpts& o, float target) {
#pragma clang fp contract(off)
  SideRow<K> ta, tb;
  ta.build(A, rA);
  tb.build(B, rB);
  const float k = ta.kpart(A) + tb.kpart(B);
  const float u = tb.vpart(B) - ta.vpart(A);
  const float nl = row_lambda<K == 0>(lam, u, k, bound, o, target);
  const float dl = nl - lam;
  ta.apply(A, -dl);
  tb.apply(B, dl);
  lam = nl;
}

// the partner lane's value (lanes 2p and 2p + 1 swap; both must be active)
__device__ __forceinline__ float pair_swap(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}

// one row on a lane pair: this lane holds body S (sg = -1: A, +1: B), its partner the other.
// k = k_A + k_B and u = v_B - v_A come out bit for bit as in row_single (a sum does not depend
// on its order of operands, and -(x - y) = y - x exactly).
template <int K>
__device__ __forceinline__ void row_pair(LBody& S, const float r[3], float& lam, float bound, const SolveOpts& o,
                                         float target, float sg) {
#pragma clang fp contract(off)
  SideRow<K> t;
  t.build(S, r);
  const float kp = t.kpart(S), vp = t.vpart(S);
  const float k = kp + pair_swap(kp);
  const float u = sg * (vp - pair_swap(vp));
  const float nl = row_lambda<K == 0>(lam, u, k, bound, o, target);
  const float dl = nl - lam;
  t.apply(S, sg * dl);
  lam = nl;
}
// one body's share of the coupling of a point's two tangent rows: (r x e_1) . I^-1 (r x e_2)
__device__ __forceinline__ float tangent_cross(const SideRow<1>& t1, const SideRow<2>& t2) {
#pragma clang fp contract(off)
  return __builtin_fmaf(t1.c1, t2.i[SideRow<1>::i1], t1.c2 * t2.i[SideRow<1>::i2]);
}

// the larger eigenvalue of the tangent block [[k1, k12], [k12, k2]]: a step 1 / kt along the slip
// overshoots in no direction of the pair
__device__ __forceinline__ float tangent_block_max(float k1, float k2, float k12) {
#pragma clang fp contract(off)
  const float h = 0.5f * (k1 - k2);
  return 0.5f * (k1 + k2) + __builtin_sqrtf(__builtin_fmaf(h, h, k12 * k12));
}

// the tangent pair of one point on the disc: both rows from the same velocities and with one
// inverse effective mass (the larger eigenvalue of the pair's block, so that the update points
// against the slip velocity), the pair of unclipped impulses projected, then both applied
__device__ __forceinline__ void cone_pair_single(LBody& A, LBody& B, const float rA[3], const float rB[3], float lam[3],
                                                 float bound) {
#pragma clang fp contract(off)
  SideRow<1> a1, b1;
  SideRow<2> a2, b2;
  a1.build(A, rA);
  b1.build(B, rB);
  a2.build(A, rA);
  b2.build(B, rB);
  const float k1 = a1.kpart(A) + b1.kpart(B), u1 = b1.vpart(B) - a1.vpart(A);
  const float k2 = a2.kpart(A) + b2.kpart(B), u2 = b2.vpart(B) - a2.vpart(A);
  const float k12 = tangent_cross(a1, a2) + tangent_cross(b1, b2);
  const float rk = __builtin_amdgcn_rcpf(tangent_block_max(k1, k2, k12));
  float l1 = __builtin_fmaf(-u1, rk, lam[1]);
  float l2 = __builtin_fmaf(-u2, rk, lam[2]);
  disc_project(l1, l2, bound);
  const float d1 = l1 - lam[1], d2 = l2 - lam[2];
  a1.apply(A, -d1);
  b1.apply(B, d1);
  a2.apply(A, -d2);
  b2.apply(B, d2);
  lam[1] = l1;
  lam[2] = l2;
}
__device__ __forceinline__ void cone_pair_lanes(LBody& S, const float r[3], float lam[3], float bound, float sg) {
#pragma clang fp contract(off)
  SideRow<1> t1;
  SideRow<2> t2;
  t1.build(S, r);
  t2.build(S, r);
  const float kp1 = t1.kpart(S), vp1 = t1.vpart(S), kp2 = t2.kpart(S), vp2 = t2.vpart(S);
  const float kx = tangent_cross(t1, t2);
  const float k1 = kp1 + pair_swap(kp1), u1 = sg * (vp1 - pair_swap(vp1));
  const float k2 = kp2 + pair_swap(kp2), u2 = sg * (vp2 - pair_swap(vp2));
  const float k12 = kx + pair_swap(kx);
  const float rk = __builtin_amdgcn_rcpf(tangent_block_max(k1, k2, k12));
  float l1 = __builtin_fmaf(-u1, rk, lam[1]);
  float l2 = __builtin_fmaf(-u2, rk, lam[2]);
  disc_project(l1, l2, bound);
  t1.apply(S, sg * (l1 - lam[1]));
  t2.apply(S, sg * (l2 - lam[2]));
  lam[1] = l1;
  lam[2] = l2;
}

// one point's rows in order: Eq. (lambda_n), then Eq. (coulomb_pgs) on t1 and t2 (or the pair
// on the disc)
__device__ __forceinline__ void solve_point(LBody& A, LBody& B, const float rA[3], const float rB[3], float lam[3],
                                            float mu, const SolveOpts& o, float target) {
  row_single<0>(A, B, rA, rB, lam[0], 0.f, o, target);
  const float bound = mu * lam[0];
  if (o.cone) {
    cone_pair_single(A, B, rA, rB, lam, bound);
  } else {
    row_single<1>(A, B, rA, rB, lam[1], bound, o, 0.f);
    row_single<2>(A, B, rA, rB, lam[2], bound, o, 0.f);
  }
}

__device__ __forceinline__ void solve_point_pair(LBody& S, const float r[3], float lam[3], float mu,
                                                 const SolveOpts& o, float target, float sg) {
  row_pair<0>(S, r, lam[0], 0.f, o, target, sg);
  const float bound = mu * lam[0];
  if (o.cone) {
    cone_pair_lanes(S, r, lam, bound, sg);
  } else {
    row_pair<1>(S, r, lam[1], bound, o, 0.f, sg);
    row_pair<2>(S, r, lam[2], bound, o, 0.f, sg);
  }
}

// what one PGS visit of a manifold reads besides the bodies: its pair, point count, friction
// coefficient and normal, and its points' lever arms and impulses, [j * 3 + k] (slots past its
// points are unused)
struct ManPoints {
  float r[12], l[12], n[3], mu;
  float tb[4];     // restitution targets of the normal rows (with the bias option)
  uint32_t ab;
  int np;
};

__device__ __forceinline__ void fetch_points(const Lds& L, int m, ManPoints& d, bool bias) {
  d.ab = L.mab[m];
  d.np = (int)(L.mmeta[m] & 15u);
  d.mu = L.mu[L.tw[d.ab >> 16]];
  // the whole record in seven 16-byte loads (slots past the manifold's points come along unused)
  const float4* rec = reinterpret_cast<const float4*>(mdev(L, m));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float4 r = rec[c], l = rec[3 + c];
    d.r[4 * c] = r.x; d.r[4 * c + 1] = r.y; d.r[4 * c + 2] = r.z; d.r[4 * c + 3] = r.w;
    d.l[4 * c] = l.x; d.l[4 * c + 1] = l.y; d.l[4 * c + 2] = l.z; d.l[4 * c + 3] = l.w;
  }
  const float4 nd = rec[6];
  d.n[0] = nd.x; d.n[1] = nd.y; d.n[2] = nd.z;
  if (bias) {
    const float4 tb = *reinterpret_cast<const float4*>(L.mtb + 4 * (size_t)m);
    d.tb[0] = tb.x; d.tb[1] = tb.y; d.tb[2] = tb.z; d.tb[3] = tb.w;
  } else {
    d.tb[0] = d.tb[1] = d.tb[2] = d.tb[3] = 0.f;
  }
}

// one PGS visit of manifold m with its data already in registers; stores the new impulses
__device__ __forceinline__ void solve_manifold_pts(const Lds& L, int m, const SolveOpts& o, ManPoints& d) {
  int a, b;
  Frame F;
  LBody A, B;
  float dAB[3];
  manifold_open(L, d.ab, d.n, a, b, F, A, B, dAB);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < d.np) {
      const float rA[3] = {d.r[3 * j], d.r[3 * j + 1], d.r[3 * j + 2]};
      const float rB[3] = {rA[0] + dAB[0], rA[1] + dAB[1], rA[2] + dAB[2]};
      solve_point(A, B, rA, rB, &d.l[3 * j], d.mu, o, d.tb[j]);
    }
  }
  store_local(L, a, F, A);
  if (b != (int)kGround) store_local(L, b, F, B);
  float4* rec = reinterpret_cast<float4*>(mdev(L, m));
#pragma unroll
  for (int c = 0; c < 3; ++c) rec[3 + c] = make_float4(d.l[4 * c], d.l[4 * c + 1], d.l[4 * c + 2], d.l[4 * c + 3]);
}

// the same visit by a lane pair: lane 2p works body A, lane 2p + 1 body B (the ground: no
// update); both hold the impulses, the first stores them
__device__ __forceinline__ void solve_manifold_pair(const Lds& L, int m, const SolveOpts& o, ManPoints& d,
                                                    bool is_b) {
  const int a = (int)(d.ab >> 16), b = (int)(d.ab & 0xffffu);
  Frame F;
  make_frame(d.n, F);
  const int me = is_b ? b : a;
  LBody S;
  load_local<true>(L, me, F, S);
  float dAB[3] = {0.f, 0.f, 0.f};
  if (b != (int)kGround) {
    float dx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dx[k] = L.x[k * L.nbp + a] - L.x[k * L.nbp + b];
    to_local(F, dx, dAB);
  }
  const float sg = is_b ? 1.f : -1.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < d.np) {
      float r[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) r[k] = is_b ? d.r[3 * j + k] + dAB[k] : d.r[3 * j + k];
      solve_point_pair(S, r, &d.l[3 * j], d.mu, o, d.tb[j], sg);
    }
  }
  store_local(L, me, F, S);
  if (!is_b) {
    float4* rec = reinterpret_cast<float4*>(mdev(L, m));
#pragma unroll
    for (int c = 0; c < 3; ++c) rec[3 + c] = make_float4(d.l[4 * c], d.l[4 * c + 1], d.l[4 * c + 2], d.l[4 * c + 3]);
  }
}

__device__ __forceinline__ void solve_manifold(const Lds& L, int m, const SolveOpts& o) {
  ManPoints d;
  fetch_points(L, m, d, o.bias);
  solve_manifold_pts(L, m, o, d);
}

// A colour of at most nthr / 2 manifolds is worked by lane pairs (pair p = tid / 2 takes
// manifolds coloff[col] + p + (nthr / 2) k); a larger one by single lanes (tid + nthr k).
__device__ __forceinline__ bool paired_colour(const Lds& L, int col, int nthr) {
  return L.coloff[col + 1] - L.coloff[col] <= (nthr >> 1);
}
__device__ __forceinline__ int colour_first(const Lds& L, int col, int tid, int nthr) {
  return L.coloff[col] + (paired_colour(L, col, nthr) ? (tid >> 1) : tid);
}

// `sweeps` PGS sweeps over the colours by the workgroup's `nthr` threads (thread `tid`).  A
// thread visits the same manifolds in the same order on every sweep, so the points of its
// next manifold are fetched from device memory while it solves the current one; one with a
// single manifold keeps it in registers.  Every thread passes the same sweeps x ncol barriers.
// (kVariants false: the literal solver, cone and bias off at compile time, so the default
// sweep loop carries none of the variants' registers)
template <bool kVariants>
__device__ __forceinline__ void pgs_sweeps_impl(const Lds& L, int sweeps, int ncol, int tid, int nthr,
                                                const SolveOpts& opts) {
  const SolveOpts o = {opts.e, kVariants && opts.cone, kVariants && opts.bias};
  int first = 0;   // the thread's first colour with a manifold (ncol: none)
  while (first < ncol && colour_first(L, first, tid, nthr) >= L.coloff[first + 1]) ++first;
  ManPoints cur, nxt;
  if (first < ncol) fetch_points(L, colour_first(L, first, tid, nthr), cur, o.bias);
  const bool is_b = tid & 1;
  for (int it = 0; it < sweeps; ++it) {
    for (int col = 0; col < ncol; ++col) {
      const bool paired = paired_colour(L, col, nthr);
      const int stride = paired ? (nthr >> 1) : nthr;
      for (int m = colour_first(L, col, tid, nthr); m < L.coloff[col + 1]; m += stride) {
        int n2 = m + stride, c2 = col;
        while (n2 >= L.coloff[c2 + 1]) {
          if (++c2 == ncol) { c2 = first; n2 = colour_first(L, first, tid, nthr); break; }
          n2 = colour_first(L, c2, tid, nthr);
        }
        const bool other = n2 != m;
        if (other) fetch_points(L, n2, nxt, o.bias);
        if (paired) solve_manifold_pair(L, m, o, cur, is_b);
        else solve_manifold_pts(L, m, o, cur);
        if (other) cur = nxt;
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ void pgs_sweeps(const Lds& L, int sweeps, int ncol, int tid, int nthr,
                                           const SolveOpts& o) {
  if (o.cone || o.bias) pgs_sweeps_impl<true>(L, sweeps, ncol, tid, nthr, o);
  else pgs_sweeps_impl<false>(L, sweeps, ncol, tid, nthr, o);
}

// One row of a visit by a lane pair from the cached share of the row (r x e_K, I^-1 (r x e_K) in
// t, the reciprocal rk of the pair's k): what row_pair computes, with the terms that do not change
// during the sweeps taken from registers.
template <int K>
__device__ __forceinline__ void row_pair_cached(LBody& S, const SideRow<K>& t, float rk, float& lam, float bound,
                                                const SolveOpts& o, float target, float sg) {
#pragma clang fp contract(off)
  const float vp = t.vpart(S);
  const float u = sg * (vp - pair_swap(vp));
  const float nl = row_lambda_rk<K == 0>(lam, u, rk, bound, o, target);
  const float dl = nl - lam;
  t.apply(S, sg * dl);
  lam = nl;
}

// The sweeps of a tower stepped by a workgroup of kNthr threads (small batches).  Lane pair
// p = tid / 2 owns colour-sorted manifold p for the whole solve: its body's share of every row
// (r x e_K, I^-1 (r x e_K)) and the rows' 1 / k are computed once, by the arithmetic of a visit,
// and kept in registers, so a visit only reads and writes its body's velocities.  The bits are
// those of pgs_sweeps (the pair mode, which single lanes match bit for bit).  A tower with more
// manifolds than lane pairs, or the disc friction variant, takes pgs_sweeps.  Every thread
// passes the same sweeps x ncol barriers.
template <int kNthr>
__device__ __forceinline__ void pgs_sweeps_lat(const Lds& L, int sweeps, int ncol, int tid, const SolveOpts& o) {
  const int nkept = L.coloff[ncol];
  if (nkept > kNthr / 2 || o.cone) {
    pgs_sweeps(L, sweeps, ncol, tid, kNthr, o);
    return;
  }
  const int p = tid >> 1;
  const bool is_b = (tid & 1) != 0;
  const bool mine = p < nkept;   // the same for both lanes of a pair
  SideRow<0> t0[4];
  SideRow<1> t1[4];
  SideRow<2> t2[4];
  float rk[4][3], lam[12], tb[4];
  Frame F;
  LBody S;
  int me = 0, np = 0, col = -1;
  float mu = 0.f, sg = 0.f;
  bool ground_me = false;
  if (mine) {
    ManPoints d;
    fetch_points(L, p, d, o.bias);
    np = d.np;
    mu = d.mu;
    const int a_ = (int)(d.ab >> 16), b_ = (int)(d.ab & 0xffffu);
    make_frame(d.n, F);
    me = is_b ? b_ : a_;
    ground_me = is_b && b_ == (int)kGround;
    load_local_g(L, me, ground_me, F, S);
    float dAB[3] = {0.f, 0.f, 0.f};
    if (b_ != (int)kGround) {
      float dx[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) dx[k] = L.x[k * L.nbp + a_] - L.x[k * L.nbp + b_];
      to_local(F, dx, dAB);
    }
    sg = is_b ? 1.f : -1.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float r[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) r[k] = is_b ? d.r[3 * j + k] + dAB[k] : d.r[3 * j + k];
      t0[j].build(S, r);
      t1[j].build(S, r);
      t2[j].build(S, r);
      if (j < np) {
        const float k0 = t0[j].kpart(S), k1 = t1[j].kpart(S), k2 = t2[j].kpart(S);
        rk[j][0] = __builtin_amdgcn_rcpf(k0 + pair_swap(k0));
        rk[j][1] = __builtin_amdgcn_rcpf(k1 + pair_swap(k1));
        rk[j][2] = __builtin_amdgcn_rcpf(k2 + pair_swap(k2));
      } else {
        rk[j][0] = rk[j][1] = rk[j][2] = 0.f;
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) lam[k] = d.l[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) tb[k] = d.tb[k];
    col = 0;
    while (L.coloff[col + 1] <= p) ++col;
  }
  for (int it = 0; it < sweeps; ++it) {
    for (int c = 0; c < ncol; ++c) {
      if (mine && c == col) {
        // the body's velocities in the frame, as load_local_g reads them
        float v[3] = {0.f, 0.f, 0.f}, w[3] = {0.f, 0.f, 0.f};
        if (!ground_me) {
          load3(L.v, L.nbp, me, v);
          load3(L.w, L.nbp, me, w);
        }
        to_local(F, v, S.v);
        to_local(F, w, S.w);
#pragma unroll
        for (int k = 0; k < 3; ++k) { S.v0[k] = S.v[k]; S.w0[k] = S.w[k]; }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (j < np) {
            row_pair_cached<0>(S, t0[j], rk[j][0], lam[3 * j], 0.f, o, tb[j], sg);
            const float bound = mu * lam[3 * j];
            row_pair_cached<1>(S, t1[j], rk[j][1], lam[3 * j + 1], bound, o, 0.f, sg);
            row_pair_cached<2>(S, t2[j], rk[j][2], lam[3 * j + 2], bound, o, 0.f, sg);
          }
        }
        store_local(L, me, F, S);
      }
      __syncthreads();
    }
  }
  if (mine && !is_b) {
    float4* rec = reinterpret_cast<float4*>(mdev(L, p));
#pragma unroll
    for (int c = 0; c < 3; ++c) rec[3 + c] = make_float4(lam[4 * c], lam[4 * c + 1], lam[4 * c + 2], lam[4 * c + 3]);
  }
}

__device__ __forceinline__ void warm_apply_manifold(const Lds& L, int m) {
  int a, b;
  Frame F;
  LBody A, B;
  float dAB[3];
  manifold_open(L, m, a, b, F, A, B, dAB);
  const int np = (int)(L.mmeta[m] & 15u);
  for (int j = 0; j < np; ++j) {
    float rA[3], rB[3], lam[3];
    load_point(L, m, j, dAB, rA, rB, lam);
    { RowTerms<0> t; t.build(A, B, rA, rB); t.apply(A, B, lam[0]); }
    { RowTerms<1> t; t.build(A, B, rA, rB); t.apply(A, B, lam[1]); }
    { RowTerms<2> t; t.build(A, B, rA, rB); t.apply(A, B, lam[2]); }
  }
  store_local(L, a, F, A);
  if (b != (int)kGround) store_local(L, b, F, B);
}

// the pair (a, b) of a record opened in its contact frame (b the ground when `ground`)
__device__ __forceinline__ void pair_open(const Lds& L, int a, int b, bool ground, const float n[3], Frame& F, LBody& A,
                                          LBody& B, float dAB[3]) {
  make_frame(n, F);
  load_local_g(L, a, false, F, A);
  load_local_g(L, b, ground, F, B);
  if (!ground) {
    float d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = L.x[k * L.nbp + a] - L.x[k * L.nbp + b];
    to_local(F, d, dAB);
  } else {
    dAB[0] = dAB[1] = dAB[2] = 0.f;
  }
}

// natural-map residual of one pair's record (np points): sum of squares and max |r| over its rows
__device__ __forceinline__ void residual_rec(const Lds& L, const float* rec, const float* tb, int a, int b, bool ground,
                                             int np, float mu, const SolveOpts& o, float& sum, float& mx) {
  Frame F;
  LBody A, B;
  float dAB[3];
  const float n[3] = {rec[24], rec[25], rec[26]};
  pair_open(L, a, b, ground, n, F, A, B, dAB);
  sum = 0.f;
  mx = 0.f;
  for (int j = 0; j < np; ++j) {
    float rA[3], rB[3], lam[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      rA[k] = rec[j * 3 + k];
      rB[k] = rA[k] + dAB[k];
      lam[k] = rec[12 + j * 3 + k];
    }
    const float bound = mu * lam[0];
    float res[3];
    {
      RowTerms<0> t;
      t.build(A, B, rA, rB);
      const float target = o.bias ? tb[j] : 0.f;
      res[0] = fminf(t.k * lam[0], t.vrel(A, B) - target);
    }
    RowTerms<1> t1;
    RowTerms<2> t2;
    t1.build(A, B, rA, rB);
    t2.build(A, B, rA, rB);
    // disc friction: one inverse effective mass, the larger eigenvalue of the tangent block
    const float kt = o.cone ? tangent_block_max(
                                  t1.k, t2.k,
                                  (t1.a1 * t2.iA[RowTerms<1>::i1] + t1.a2 * t2.iA[RowTerms<1>::i2]) +
                                      (t1.b1 * t2.iB[RowTerms<1>::i1] + t1.b2 * t2.iB[RowTerms<1>::i2]))
                            : 0.f;
    const float k1 = o.cone ? kt : t1.k, k2 = o.cone ? kt : t2.k;
    float cl1 = lam[1] - t1.vrel(A, B) * __builtin_amdgcn_rcpf(k1);
    float cl2 = lam[2] - t2.vrel(A, B) * __builtin_amdgcn_rcpf(k2);
    if (o.cone) {
      disc_project(cl1, cl2, bound);
    } else {
      cl1 = fminf(fmaxf(cl1, -bound), bound);
      cl2 = fminf(fmaxf(cl2, -bound), bound);
    }
    res[1] = k1 * (lam[1] - cl1);
    res[2] = k2 * (lam[2] - cl2);
#pragma unroll
    for (int r = 0; r < 3; ++r) { sum += res[r] * res[r]; mx = fmaxf(mx, fabsf(res[r])); }
  }
}

// natural-map residual of one manifold: sum of squares and max |r| over its rows
__device__ __forceinline__ void residual_manifold(const Lds& L, int m, float mu, const SolveOpts& o, float& sum,
                                                  float& mx) {
  const uint32_t ab = L.mab[m];
  const int b = (int)(ab & 0xffffu);
  residual_rec(L, mdev(L, m), L.mtb + 4 * (size_t)m, (int)(ab >> 16), b, b == (int)kGround, (int)(L.mmeta[m] & 15u),
               mu, o, sum, mx);
}

// ------------------------------------------------------------------------------------------------
// learned warm start: contact features, initial impulses from the network's outputs
// ------------------------------------------------------------------------------------------------
// The 24 network inputs of point j of colour-sorted manifold m, before the solve:
// F (x_B - x_A), q_A^-1 q_B (w >= 0), world normal, depth, mu, previous impulses (ml holds them
// after the key lookup) in the outputs' units lambda_d k_d / (|g| dt) with this step's k,
// F r_A, F r_B, F (relative velocity of B with respect to A at the point).  The ground is a
// body at (x_A, y_A, 0) with the identity orientation.
__device__ __forceinline__ void point_features(const Lds& L, int m, int j, float gdt, float f[mlp::kFeat]) {
  const int nb = L.nbp;
  const uint32_t ab = L.mab[m];
  const int ia = (int)(ab >> 16), ib = (int)(ab & 0xffffu);
  const bool ground = ib == (int)kGround;
  const float n[3] = {mdev(L, m)[24], mdev(L, m)[25], mdev(L, m)[26]};
  Frame F;
  make_frame(n, F);
  float xa[3], xb[3], d[3], dl[3];
  load3(L.x, nb, ia, xa);
  if (ground) { xb[0] = xa[0]; xb[1] = xa[1]; xb[2] = 0.f; }
  else load3(L.x, nb, ib, xb);
#pragma unroll
  for (int k = 0; k < 3; ++k) d[k] = xb[k] - xa[k];
  to_local(F, d, dl);
  f[0] = dl[0]; f[1] = dl[1]; f[2] = dl[2];
  const float aw = L.q[ia], ax = -L.q[nb + ia], ay = -L.q[2 * nb + ia], az = -L.q[3 * nb + ia];
  float bw = 1.f, bx = 0.f, by = 0.f, bz = 0.f;
  if (!ground) { bw = L.q[ib]; bx = L.q[nb + ib]; by = L.q[2 * nb + ib]; bz = L.q[3 * nb + ib]; }
  const float rw = aw * bw - ax * bx - ay * by - az * bz;
  const float rx = aw * bx + ax * bw + ay * bz - az * by;
  const float ry = aw * by - ax * bz + ay * bw + az * bx;
  const float rz = aw * bz + ax * by - ay * bx + az * bw;
  const float sg = rw < 0.f ? -1.f : 1.f;
  f[3] = sg * rw; f[4] = sg * rx; f[5] = sg * ry; f[6] = sg * rz;
  f[7] = n[0]; f[8] = n[1]; f[9] = n[2];
  f[10] = mdev(L, m)[27];
  f[11] = L.mu[L.tw[ia]];
  float rA[3], rB[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    rA[k] = mdev(L, m)[j * 3 + k];
    rB[k] = rA[k] - dl[k];
    f[15 + k] = rA[k];
    f[18 + k] = rB[k];
  }
  LBody A, B;
  load_local<false>(L, ia, F, A);
  load_local<true>(L, ib, F, B);
  {
    // the solver's own rows (rB for the ground only matters through the ground's zero terms)
    float kk[3];
    RowTerms<0> t0;
    RowTerms<1> t1;
    RowTerms<2> t2;
    t0.build(A, B, rA, rB);
    t1.build(A, B, rA, rB);
    t2.build(A, B, rA, rB);
    kk[0] = t0.k; kk[1] = t1.k; kk[2] = t2.k;
#pragma unroll
    for (int k = 0; k < 3; ++k) f[12 + k] = mdev(L, m)[12 + j * 3 + k] * kk[k] / gdt;
  }
  float ua[3], ub[3];
  cross3(A.w, rA, ua);
  cross3(B.w, rB, ub);
#pragma unroll
  for (int k = 0; k < 3; ++k) f[21 + k] = (B.v[k] + ub[k]) - (A.v[k] + ua[k]);
}

// Initial impulses of manifold m from s = network output + previous dimensionless impulses (held
// in ml), applied like solver impulses: lambda_n = max(0, s_n) |g| dt / k_n,
// lambda_t = clip(s_t |g| dt / k_t, +-mu lambda_n).
__device__ __forceinline__ void learned_apply_manifold(const Lds& L, int m, float mu, float gdt, bool cone) {
  int a, b;
  Frame F;
  LBody A, B;
  float dAB[3];
  manifold_open(L, m, a, b, F, A, B, dAB);
  const int np = (int)(L.mmeta[m] & 15u);
  for (int j = 0; j < np; ++j) {
    float rA[3], rB[3], y[3];
    load_point(L, m, j, dAB, rA, rB, y);
    RowTerms<0> t0;
    RowTerms<1> t1;
    RowTerms<2> t2;
    t0.build(A, B, rA, rB);
    t1.build(A, B, rA, rB);
    t2.build(A, B, rA, rB);
    const float ln = fmaxf(y[0], 0.f) * gdt / t0.k;
    const float bound = mu * ln;
    float l1 = y[1] * gdt / t1.k, l2 = y[2] * gdt / t2.k;
    if (cone) {
      disc_project(l1, l2, bound);
    } else {
      l1 = fminf(fmaxf(l1, -bound), bound);
      l2 = fminf(fmaxf(l2, -bound), bound);
    }
    t0.apply(A, B, ln);
    t1.apply(A, B, l1);
    t2.apply(A, B, l2);
    mdev(L, m)[12 + j * 3 + 0] = ln;
    mdev(L, m)[12 + j * 3 + 1] = l1;
    mdev(L, m)[12 + j * 3 + 2] = l2;
  }
  store_local(L, a, F, A);
  if (b != (int)kGround) store_local(L, b, F, B);
}

// k and the solved impulses of manifold m into its points' feature records
__device__ __forceinline__ void record_solution(const Lds& L, int m, float* rec) {
  int a, b;
  Frame F;
  LBody A, B;
  float dAB[3];
  manifold_open(L, m, a, b, F, A, B, dAB);
  const int np = (int)(L.mmeta[m] & 15u);
  for (int j = 0; j < np; ++j) {
    float rA[3], rB[3], lam[3];
    load_point(L, m, j, dAB, rA, rB, lam);
    RowTerms<0> t0;
    RowTerms<1> t1;
    RowTerms<2> t2;
    t0.build(A, B, rA, rB);
    t1.build(A, B, rA, rB);
    t2.build(A, B, rA, rB);
    float* r = rec + j * kFeatRecord;
    r[24] = t0.k; r[25] = t1.k; r[26] = t2.k;
    r[27] = lam[0]; r[28] = lam[1]; r[29] = lam[2];
  }
}

// Natural-map residual of each tower (RMS over its rows and max |r|) into tres: partial sums per
// canonical pair in psum / pmax (which may alias cab / cpos: each entry is read before it is
// written), then each tower's contiguous canonical range.  With `only`, towers whose flag is
// clear keep their residual.
// Each canonical pair's residual terms (pairs first, first + stride, ...); psum and pmax may
// alias the canonical lists (a pair's entry is read before it is overwritten, by one thread).
__device__ __forceinline__ void residual_parts(const Lds& L, int nman, int first, int stride, float* psum, float* pmax,
                                               const uint32_t* only, const SolveOpts& o) {
  for (int p = first; p < nman; p += stride) {
    const int m = L.cpos[p];
    float sum = 0.f, mx = 0.f;
    if (m >= 0) {
      const int t = L.tw[L.mab[m] >> 16];
      if (!only || only[t]) residual_manifold(L, m, L.mu[t], o, sum, mx);
    }
    psum[p] = sum;
    pmax[p] = mx;
  }
}

// The towers' residuals from the pairs' terms (fixed summation order); `parts` false when the
// terms are already in psum and pmax.
__device__ __forceinline__ void tower_residuals(const Lds& L, int nman, int nt, int lane, float* psum, float* pmax,
                                const uint32_t* only, const SolveOpts& o, bool parts = true) {
  if (parts) {
    residual_parts(L, nman, lane, kWave, psum, pmax, only, o);
    wave_sync();
  }
  if (nt == 1) {
    // one tower (an island): the whole wave reduces its range
    if (!only || only[0]) {
      float sum = 0.f, mx = 0.f;
      for (int p = L.tc0[0] + lane; p < L.tc1[0]; p += kWave) {
        sum += psum[p];
        mx = fmaxf(mx, pmax[p]);
      }
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        sum += __shfl_xor(sum, d);
        mx = fmaxf(mx, __shfl_xor(mx, d));
      }
      const int rows = 3 * L.tpts[0];
      if (lane == 0) {
        L.tres[0] = rows ? sqrtf(sum / (float)rows) : 0.f;
        L.tres[1] = mx;
      }
    }
    return;
  }
  for (int t = lane; t < nt; t += kWave) {
    if (only && !only[t]) continue;
    float sum = 0.f, mx = 0.f;
    for (int p = L.tc0[t]; p < L.tc1[t]; ++p) {
      sum += psum[p];
      mx = fmaxf(mx, pmax[p]);
    }
    const int rows = 3 * L.tpts[t];
    L.tres[2 * t] = rows ? sqrtf(sum / (float)rows) : 0.f;
    L.tres[2 * t + 1] = mx;
  }
}

// Contact manifolds of the canonical pairs p = first, first + stride, ... < nman, written into
// their colour-sorted slots (points, normal, depth, and the previous step's impulses when kept).
// Pairs are independent, so any number of threads can share the list.
// The contact points of colliding pair (i, j) (j the ground when `ground`): lever arms r_A in the
// contact frame into rec[0..12), the normal (from i to j) and depth; returns the point count and
// the points' slots (4 bits each).  The ground: Sec. "Narrowphase" reading R18; two boxes: the
// SAT normal and the silhouette clip (R15, R16), or reference-face clipping (manifold_mode 1).
// sat: the narrowphase's normal and depth of the pair (n [3], depth), or null to take them again
// here (both come from sat_boxes on the same inputs)
template <bool kExt>
__device__ __forceinline__ int manifold_geometry(const Lds& L, int i, int j, bool ground, int manifold_mode, float* rec,
                                                 float n[3], float& depth, uint32_t& slots, const float* sat) {
  const int NB = L.nbp;
  float t1[3], rA[4][3];
  uint32_t used = 0u;
  depth = 0.f;
  slots = 0u;
  int npts = 0;
  float R[9], he[3];
  body_R(L, i, R);
  load3(L.he, NB, i, he);
  if (ground) {
    // vertices below the ground: the four deepest (ties: lower vertex index), in index order
    const float xz = L.x[2 * NB + i];
    float vz[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float s0 = (k & 1) ? he[0] : -he[0], s1 = (k & 2) ? he[1] : -he[1], s2 = (k & 4) ? he[2] : -he[2];
      vz[k] = xz + (R[6] * s0 + R[7] * s1 + R[8] * s2);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int rank = 0;
#pragma unroll
      for (int q = 0; q < 8; ++q) rank += (vz[q] < 0.f) && (vz[q] < vz[k] || (vz[q] == vz[k] && q < k));
      if ((vz[k] < 0.f) && rank < 4) {
        const float s0 = (k & 1) ? he[0] : -he[0], s1 = (k & 2) ? he[1] : -he[1], s2 = (k & 4) ? he[2] : -he[2];
        const float rx = R[0] * s0 + R[1] * s1 + R[2] * s2;
        const float ry = R[3] * s0 + R[4] * s1 + R[5] * s2;
        const float rz = R[6] * s0 + R[7] * s1 + R[8] * s2;
        // r_A = (rx, ry, (rz - xz)/2) in the frame n = -z, t1 = x, t2 = -y
        rec[npts * 3 + 0] = 0.5f * (xz - rz);
        rec[npts * 3 + 1] = rx;
        rec[npts * 3 + 2] = -ry;
        slots |= (uint32_t)k << (4 * npts);
        depth = fmaxf(depth, -vz[k]);
        ++npts;
      }
    }
    n[0] = 0.f; n[1] = 0.f; n[2] = -1.f;
    t1[0] = 1.f; t1[1] = 0.f; t1[2] = 0.f;
  } else {
    float RB[9], heB[3], d[3];
    body_R(L, j, RB);
    load3(L.he, NB, j, heB);
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = L.x[k * NB + j] - L.x[k * NB + i];
    if (kExt && manifold_mode) {
      int ax = 0;
      sat_boxes<true>(R, he, RB, heB, d, n, depth, &ax);   // the narrowphase's inputs: it collides
      used = manifold_refface(R, he, RB, heB, d, n, ax, t1, rA);
      if (!used) used = manifold_boxes(R, he, RB, heB, d, n, t1, rA);
    } else {
      if (sat) {
        const float4 nd = *reinterpret_cast<const float4*>(sat);
        n[0] = nd.x; n[1] = nd.y; n[2] = nd.z;
        depth = nd.w;
      } else {
        sat_boxes(R, he, RB, heB, d, n, depth);
      }
      used = manifold_boxes(R, he, RB, heB, d, n, t1, rA);
    }
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
      if ((used >> s2) & 1u) {
#pragma unroll
        for (int k = 0; k < 3; ++k) rec[npts * 3 + k] = rA[s2][k];
        slots |= (uint32_t)s2 << (4 * npts);
        ++npts;
      }
  }
  return npts;
}

// The restitution targets of the pair's normal rows (restitution_bias): tb[q] for its points,
// -e v_n- from the velocities before any impulse of the step, in the contact frame (n is its first
// axis), for a point approaching faster than twice |g| dt (a resting contact approaches at about
// |g| dt per step and does not bounce).
__device__ __forceinline__ void bias_targets(const Lds& L, int i, int j, bool ground, const float* rec, float* tb,
                                             int npts, const float n[3], const float g[3], float dt, float e) {
  const int NB = L.nbp;
  const float vth = 2.f * sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]) * dt;
  Frame F;
  make_frame(n, F);
  float tmp[3], vA[3], wA[3], vB[3] = {0.f, 0.f, 0.f}, wB[3] = {0.f, 0.f, 0.f}, dAB[3] = {0.f, 0.f, 0.f};
  load3(L.v, NB, i, tmp); to_local(F, tmp, vA);
  load3(L.w, NB, i, tmp); to_local(F, tmp, wA);
  if (!ground) {
    load3(L.v, NB, j, tmp); to_local(F, tmp, vB);
    load3(L.w, NB, j, tmp); to_local(F, tmp, wB);
#pragma unroll
    for (int k = 0; k < 3; ++k) tmp[k] = L.x[k * NB + i] - L.x[k * NB + j];
    to_local(F, tmp, dAB);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float tgt = 0.f;
    if (q < npts) {
      const float ra[3] = {rec[3 * q], rec[3 * q + 1], rec[3 * q + 2]};
      const float rb[3] = {ra[0] + dAB[0], ra[1] + dAB[1], ra[2] + dAB[2]};
      const float vn = (vB[0] + (wB[1] * rb[2] - wB[2] * rb[1])) - (vA[0] + (wA[1] * ra[2] - wA[2] * ra[1]));
      tgt = vn < -vth ? -e * vn : 0.f;
    }
    tb[q] = tgt;
  }
}

template <bool kExt>
__device__ __forceinline__ void build_manifolds(const Lds& L, const StepArgs& a, int first, int stride, int nman,
                                                bool keep_prev) {
  const int PC = L.pc;
  const int nprev = L.scal[4];
  for (int p = first; p < nman; p += stride) {
    const int sidx = L.cpos[p];
    if (sidx < 0) continue;
    const uint32_t code = L.cab[p];
    const int i = (int)(code >> 16), j = (int)(code & 0xffffu);
    float n[3], depth;
    uint32_t slots;
    const int npts = manifold_geometry<kExt>(L, i, j, j == (int)kGround, a.manifold_mode, mdev(L, sidx), n, depth, slots,
                                             L.msat + 4 * (size_t)p);
    // warm start: previous step's impulses of the same (pair, slot) if the normal barely turned
    int found = -1;
    if (keep_prev && nprev > 0) {
      int lo = 0, hi = nprev - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const uint32_t kk = L.pkey[mid];
        if (kk == code) { found = mid; break; }
        if (kk < code) lo = mid + 1; else hi = mid - 1;
      }
      if (found >= 0) {
        const float pn[3] = {L.pnrm[found], L.pnrm[PC + found], L.pnrm[2 * PC + found]};
        if (!(dot3(pn, n) > 0.95f)) found = -1;
      }
    }
    for (int q = 0; q < npts; ++q) {
      float l0 = 0.f, l1 = 0.f, l2 = 0.f;
      if (found >= 0) {
        const uint32_t ps = L.pslot[found];
        const int pnp = (int)(ps & 15u);
        const uint32_t sq = (slots >> (4 * q)) & 15u;
        for (int r = 0; r < pnp; ++r)
          if (((ps >> (4 + 4 * r)) & 15u) == sq) {
            l0 = L.plam[(r * 3 + 0) * PC + found];
            l1 = L.plam[(r * 3 + 1) * PC + found];
            l2 = L.plam[(r * 3 + 2) * PC + found];
          }
      }
      mdev(L, sidx)[12 + q * 3 + 0] = l0;
      mdev(L, sidx)[12 + q * 3 + 1] = l1;
      mdev(L, sidx)[12 + q * 3 + 2] = l2;
    }
    if (kExt && a.restitution_bias)
      bias_targets(L, i, j, j == (int)kGround, mdev(L, sidx), L.mtb + 4 * (size_t)sidx, npts, n, a.g, a.dt, a.restitution);
    L.mab[sidx] = code;
    L.mmeta[sidx] = (uint32_t)npts | (slots << 12);
    mdev(L, sidx)[27] = depth;
    if (keep_prev) L.mcanon[sidx] = p;
#pragma unroll
    for (int k = 0; k < 3; ++k) mdev(L, sidx)[24 + k] = n[k];
    const int ti = L.tw[i];
    atomicAdd(&L.tcnt[ti * 4 + 1], 1u);
    atomicAdd(&L.tcnt[ti * 4 + 2], (uint32_t)npts);
    atomicAdd(&L.tpts[ti], npts);
  }
}

// Semi-implicit integration of dynamic body i over dt (Eq. (newton_euler), Eq. (quat_int), R1, R4):
// x += dt v; q' = normalise(q + dt/2 [0, w] q); w' = I_w(q')^-1 I_w(q) w.  Returns false when the
// new state is not finite (it is stored all the same).
__device__ __forceinline__ bool integrate_body(const Lds& L, int i, float m, float dt) {
  const int NB = L.nbp;
  float xv[3], vv[3], wv[3], R[9], Ib[3], iIb[3];
  load3(L.x, NB, i, xv);
  load3(L.v, NB, i, vv);
  load3(L.w, NB, i, wv);
  body_R(L, i, R);
  inv_body_inertia(L, i, m, iIb);
#pragma unroll
  for (int k = 0; k < 3; ++k) { xv[k] += dt * vv[k]; Ib[k] = 1.f / iIb[k]; }
  // L = R Ib R^T w
  float bw[3], Lw[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) bw[k] = (R[k] * wv[0] + R[3 + k] * wv[1] + R[6 + k] * wv[2]) * Ib[k];
#pragma unroll
  for (int r = 0; r < 3; ++r) Lw[r] = R[3 * r] * bw[0] + R[3 * r + 1] * bw[1] + R[3 * r + 2] * bw[2];
  float qw = L.q[i], qx = L.q[NB + i], qy = L.q[2 * NB + i], qz = L.q[3 * NB + i];
  const float hd = 0.5f * dt;
  const float dw = -(wv[0] * qx + wv[1] * qy + wv[2] * qz);
  const float dx = wv[0] * qw + (wv[1] * qz - wv[2] * qy);
  const float dy = wv[1] * qw + (wv[2] * qx - wv[0] * qz);
  const float dz = wv[2] * qw + (wv[0] * qy - wv[1] * qx);
  qw += hd * dw; qx += hd * dx; qy += hd * dy; qz += hd * dz;
  const float il = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  qw *= il; qx *= il; qy *= il; qz *= il;
  quat_rot(qw, qx, qy, qz, R);
  float bl[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) bl[k] = (R[k] * Lw[0] + R[3 + k] * Lw[1] + R[6 + k] * Lw[2]) * iIb[k];
#pragma unroll
  for (int r = 0; r < 3; ++r) wv[r] = R[3 * r] * bl[0] + R[3 * r + 1] * bl[1] + R[3 * r + 2] * bl[2];
  bool finite = isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz);
#pragma unroll
  for (int k = 0; k < 3; ++k) finite = finite && isfinite(xv[k]) && isfinite(vv[k]) && isfinite(wv[k]);
  store3(L.x, NB, i, xv);
  store3(L.w, NB, i, wv);
  L.q[i] = qw; L.q[NB + i] = qx; L.q[2 * NB + i] = qy; L.q[3 * NB + i] = qz;
  return finite;
}

// Baumgarte position correction of one colliding pair (Eq. (baumgarte), reading R19), from its
// record's depth and normal: x_A -= beta m_A^-1 c n, x_B += beta m_B^-1 c n with
// c = max(0, depth - slop) / (m_A^-1 + m_B^-1), dynamic bodies only.
__device__ __forceinline__ void baumgarte_pair(const Lds& L, int i, int j, bool ground, const float* rec, float beta,
                                               float slop) {
  const int NB = L.nbp;
  const bool di = (L.flag[i] & kDynamic) != 0;
  const bool dj = !ground && (L.flag[j] & kDynamic);
  const float ia = di ? L.invm[i] : 0.f, ib = dj ? L.invm[j] : 0.f;
  float corr = rec[27] - slop;
  if (ia + ib <= 0.f || corr <= 0.f) return;
  corr /= (ia + ib);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float nk = rec[24 + k];
    if (di) L.x[k * NB + i] -= beta * ia * corr * nk;
    if (dj) L.x[k * NB + j] += beta * ib * corr * nk;
  }
}

// Island broadphase (bodies in device memory, one tower per pack).
// The candidates of the 64 bodies i = i0 + lane, each lane's in canonical order (j
// ascending, the ground last): counted, and the first kCandPerBody written from out + off.  Windows are visited
// in order; a window near none of the 64 is skipped, and a near one is loaded into
// registers (lane l: body 64 w + l) and broadcast body by body with readlane, so the
// tests of one lane wait on no memory.
__device__ __forceinline__ int island_walk(const Lds& L, float margin, int nb, int nwin, int i0, int lane, uint32_t* out,
                                           int off) {
  const int NB = L.nbp;
  const float slack = margin * 1.01f + 1e-6f;   // a filter: wider than the pair test
  constexpr int lim = kCandPerBody;
  const int i = i0 + lane;
  const uint32_t fi = i < nb ? L.flag[i] : 0u;
  const bool act = (fi & kActive) != 0;
  const bool dyni = (fi & kDynamic) != 0;
  float xi[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
  if (act) {
#pragma unroll
    for (int k = 0; k < 3; ++k) { xi[k] = L.x[k * NB + i]; hi[k] = L.hm[k * NB + i]; }
  }
  int c = 0;
  const int w0 = i0 / kWave;
  for (int wb0 = w0 - w0 % kWave; wb0 < nwin; wb0 += kWave) {
    // lane l holds the box of window wb0 + l
    float blo[3], bhi[3];
    const bool inw = wb0 + lane < nwin;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      blo[k] = inw ? L.wbox[6 * (wb0 + lane) + k] : 0.f;
      bhi[k] = inw ? L.wbox[6 * (wb0 + lane) + 3 + k] : 0.f;
    }
    for (int w = max(w0, wb0); w < min(nwin, wb0 + kWave); ++w) {
      // broadcasts first, then branch-free tests (& rather than &&: no masked regions)
      float lo[3], hb[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        lo[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(blo[k]), w - wb0));
        hb[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bhi[k]), w - wb0));
      }
      bool near = act;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        near = ((int)near & (int)(xi[k] - hi[k] <= hb[k] + slack) & (int)(xi[k] + hi[k] + slack >= lo[k])) != 0;
      if (!__any(near)) continue;
      const int jl = w * kWave + lane;
      const bool inj = jl < nb;
      float xj[3], hj[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        xj[k] = inj ? L.x[k * NB + jl] : 0.f;
        hj[k] = inj ? L.hm[k * NB + jl] : 0.f;
      }
      const uint32_t fj = inj ? L.flag[jl] : 0u;
      const int jn = min(kWave, nb - w * kWave);
      for (int jj = 0; jj < jn; ++jj) {
        const int j = w * kWave + jj;
        const uint32_t f = __builtin_amdgcn_readlane(fj, jj);
        float d[3], h[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          d[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(xj[k]), jj));
          h[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hj[k]), jj));
        }
        const int hitm = (int)near & (int)(j > i) & (int)((f & kActive) != 0) &
                         ((int)dyni | (int)((f & kDynamic) != 0)) &
                         (int)(fabsf(xi[0] - d[0]) <= hi[0] + h[0] + margin) &
                         (int)(fabsf(xi[1] - d[1]) <= hi[1] + h[1] + margin) &
                         (int)(fabsf(xi[2] - d[2]) <= hi[2] + h[2] + margin);
        const bool hit = hitm != 0;
        if (hit) {
          if (c < lim) out[off + c] = ((uint32_t)i << 16) | (uint32_t)j;
          ++c;
        }
      }
    }
  }
  if (act && dyni && (xi[2] - hi[2] <= margin)) {
    if (c < lim) out[off + c] = ((uint32_t)i << 16) | kGround;
    ++c;
  }
  return c;
}

// Walk rounds i0 = 64 (first + k stride) of the island broadphase: each body's candidates into its
// own kCandPerBody slots and their count (capped) into the colouring lane masks, which are
// unused until the colouring.  A wave may be one of several sharing the rounds (first, stride in
// waves): the bodies, slots and counts of distinct rounds are distinct.
__device__ __forceinline__ void island_walk_rounds(const Lds& L, float margin, int nb, int first, int stride, int lane) {
  const int nwin = (nb + kWave - 1) / kWave;
  bool over = false;
  for (int i0 = first * kWave; i0 < nb; i0 += stride * kWave) {
    const int i = i0 + lane;
    const int c = island_walk(L, margin, nb, nwin, i0, lane, L.cslot, i * kCandPerBody);
    over = over || c > kCandPerBody;
    if (i < nb) L.lmlo[i] = (uint32_t)min(c, kCandPerBody);
  }
  if (__any(over) && lane == 0) atomicOr((uint32_t*)&L.scal[3], kErrCand);
}

// The learned warm start's network inputs, initial impulses and feature records for chunks of 16
// manifolds x 4 point slots (lane = 4 (m - m0) + j), chunks first, first + stride, ... of the
// colour-sorted list; xs is the calling wave's staging rows (unused for records alone).
__device__ __forceinline__ void learned_chunks(const Lds& L, const StepArgs& a, int nkept, int slot0, float gdt,
                                               bool learned, bool rec, int first, int stride, int lane,
                                               uint32_t* xs) {
  const uint4* net = (const uint4*)a.mlp;
  for (int m0 = first * (kWave / 4); m0 < nkept; m0 += stride * (kWave / 4)) {
    const int m = m0 + (lane >> 2), j = lane & 3;
    const bool valid = m < nkept && j < (int)(L.mmeta[m] & 15u);
    float f[mlp::kFeat];
    if (valid) point_features(L, m, j, gdt, f);
    else
#pragma unroll
      for (int k = 0; k < mlp::kFeat; ++k) f[k] = 0.f;
    if (rec && valid) {
      float* o = a.feat_out + ((size_t)(slot0 + m) * 4 + j) * kFeatRecord;
#pragma unroll
      for (int k = 0; k < mlp::kFeat; ++k) o[k] = f[k];
    }
    if (learned) {
      // the network predicts the change from the previous dimensionless impulses
      float* prevd = reinterpret_cast<float*>(xs + kWave * mlp::kRowWords);
      mlp::stage_row(net, f, xs + lane * mlp::kRowWords);
#pragma unroll
      for (int k = 0; k < 3; ++k) prevd[3 * lane + k] = f[12 + k];
      wave_sync();
      mlp::f32x4 y[4];
      mlp::infer_chunk(net, xs, lane, y);
      if (lane < 16) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int row = 16 * t + lane, mm = m0 + (row >> 2), jj = row & 3;
          if (mm < nkept && jj < (int)(L.mmeta[mm] & 15u))
#pragma unroll
            for (int k = 0; k < 3; ++k) mdev(L, mm)[12 + jj * 3 + k] = y[t][k] + prevd[3 * row + k];
        }
      }
      wave_sync();
    }
  }
}

// ------------------------------------------------------------------------------------------------
// episodes (Sec. "Stability Detection and Collapse"): at the end of each step, one lane per tower
// ------------------------------------------------------------------------------------------------
// The support polygon of Eq. (stability): the horizontal corners of every active block whose lowest
// point is within eps of the ground, staged in scratch (16 floats per body of the tower), wrapped
// counter-clockwise from the leftmost-lowest corner (gift wrapping: the next vertex leaves no
// corner to its right; of collinear corners the farthest); the margin is the smallest signed
// distance of the centre of mass to the wrapped edges (positive inside; -inf with fewer than three
// vertices).
__device__ __forceinline__ float support_margin(const Lds& L, int b0, int b1, float eps, float cx, float cy,
                                                float* pts, int& nhull) {
  const int NB = L.nbp;
  int n = 0;
  for (int i = b0; i < b1; ++i) {
    if ((L.flag[i] & (kActive | kDynamic)) != (kActive | kDynamic)) continue;
    float R[9];
    body_R(L, i, R);
    const float he0 = L.he[i], he1 = L.he[NB + i], he2 = L.he[2 * NB + i];
    const float hz = fabsf(R[6]) * he0 + fabsf(R[7]) * he1 + fabsf(R[8]) * he2;
    if (!(L.x[2 * NB + i] - hz <= eps)) continue;
    const float xi = L.x[i], yi = L.x[NB + i];
    for (int c = 0; c < 8; ++c) {
      const float s0 = (c & 1) ? he0 : -he0, s1 = (c & 2) ? he1 : -he1, s2 = (c & 4) ? he2 : -he2;
      pts[2 * n] = xi + (R[0] * s0 + R[1] * s1 + R[2] * s2);
      pts[2 * n + 1] = yi + (R[3] * s0 + R[4] * s1 + R[5] * s2);
      ++n;
    }
  }
  nhull = 0;
  if (n == 0) return -INFINITY;
  int start = 0;
  for (int k = 1; k < n; ++k)
    if (pts[2 * k] < pts[2 * start] || (pts[2 * k] == pts[2 * start] && pts[2 * k + 1] < pts[2 * start + 1])) start = k;
  const float sx = pts[2 * start], sy = pts[2 * start + 1];
  float ax = sx, ay = sy;
  float margin = INFINITY;
  for (int it = 0; it <= n; ++it) {
    int nx = -1;
    float bx = 0.f, by = 0.f, bd = 0.f;
    for (int k = 0; k < n; ++k) {
      const float px = pts[2 * k], py = pts[2 * k + 1];
      if (px == ax && py == ay) continue;
      const float d2 = (px - ax) * (px - ax) + (py - ay) * (py - ay);
      if (nx < 0) { nx = k; bx = px; by = py; bd = d2; continue; }
      const float c = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
      if (c < 0.f || (c == 0.f && d2 > bd)) { nx = k; bx = px; by = py; bd = d2; }
    }
    if (nx < 0) break;                      // every corner at one point
    const float len = sqrtf(bd);
    margin = fminf(margin, ((bx - ax) * (cy - ay) - (by - ay) * (cx - ax)) / len);
    ++nhull;
    ax = bx;
    ay = by;
    if (ax == sx && ay == sy) break;
  }
  return nhull >= 3 ? margin : -INFINITY;
}

// The criteria of Eq. (collapse) for each tower of the pack at the end of step `step`, and the
// episode rules: a collapse is declared on the first step whose end state meets all three (the
// imbalance keeps minus the margin of the step before); afterwards the tower is held once its
// kinetic energy falls below ek_rest or ep_rest_steps steps have passed.  Sums run over the
// tower's bodies in order (deterministic).  `scratch` holds 16 floats per body of the pack.
__device__ __forceinline__ void episode_update(const Lds& L, const StepArgs& a, int gt0, int gb0, int nt, int lane,
                                               int64_t step, float* scratch) {
  const int NB = L.nbp, CAP = a.cap;
  for (int t = lane; t < nt; t += kWave) {
    uint32_t* st = a.ep_state + (size_t)(gt0 + t) * kEpisodeWords;
    uint32_t flags = st[kEpFlags];
    if (flags & kEpDone) continue;
    const int b0 = L.tb0[t], b1 = L.tb1[t];
    float ek = 0.f, dxmax = 0.f, rzz = 1.f, msum = 0.f, cx = 0.f, cy = 0.f;
    bool cd = false;
    for (int i = b0; i < b1; ++i) {
      if ((L.flag[i] & (kActive | kDynamic)) != (kActive | kDynamic)) continue;
      const float m = a.mass[gb0 + i];
      float R[9];
      body_R(L, i, R);
      const float l = 2.f * L.he[i], wd = 2.f * L.he[NB + i], hh = 2.f * L.he[2 * NB + i];
      const float I0 = m / 12.f * (wd * wd + hh * hh), I1 = m / 12.f * (l * l + hh * hh),
                  I2 = m / 12.f * (l * l + wd * wd);
      float v[3], w[3];
      load3(L.v, NB, i, v);
      load3(L.w, NB, i, w);
      const float wb0 = R[0] * w[0] + R[3] * w[1] + R[6] * w[2];
      const float wb1 = R[1] * w[0] + R[4] * w[1] + R[7] * w[2];
      const float wb2 = R[2] * w[0] + R[5] * w[1] + R[8] * w[2];
      ek += 0.5f * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      ek += 0.5f * (I0 * wb0 * wb0 + I1 * wb1 * wb1 + I2 * wb2 * wb2);
      float d2 = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float d = L.x[k * NB + i] - a.ep_x0[k * CAP + gb0 + i];
        d2 += d * d;
      }
      const float dn = sqrtf(d2);
      dxmax = fmaxf(dxmax, dn);
      cd = cd || dn > a.ep_fd * l;
      rzz = fminf(rzz, R[8]);
      msum += m;
      cx += m * L.x[i];
      cy += m * L.x[NB + i];
    }
    if (msum > 0.f) { cx /= msum; cy /= msum; }
    int nhull = 0;
    const float margin = support_margin(L, b0, b1, a.ep_eps, cx, cy, scratch + 16 * b0, nhull);
    const bool ck = ek > a.ep_ek_collapse, ct = rzz < a.ep_cos_theta;
    st[kEpSupport] = (uint32_t)nhull;
    st[kEpEk] = __float_as_uint(ek);
    st[kEpDx] = __float_as_uint(dxmax);
    st[kEpTheta] = __float_as_uint(acosf(fmaxf(rzz, -1.f)));
    st[kEpMargin] = __float_as_uint(margin);
    st[kEpComX] = __float_as_uint(cx);
    st[kEpComY] = __float_as_uint(cy);
    if (!(flags & kEpCollapsed)) {
      if (cd && ck && ct) {
        flags |= kEpCollapsed;
        st[kEpCollapseStep] = (uint32_t)(int32_t)step;
        L.tfz[t] |= 4u;                     // no further push or withdrawal
      } else {
        st[kEpImbalance] = __float_as_uint(-margin);
      }
    }
    if (flags & kEpCollapsed) {
      const int64_t since = step - (int64_t)(int32_t)st[kEpCollapseStep];
      if (ek < a.ep_ek_rest) {
        flags |= kEpDone;
        st[kEpRestStep] = (uint32_t)(int32_t)step;
      } else if (since >= a.ep_rest_steps) {
        flags |= kEpDone;
        st[kEpRestStep] = (uint32_t)(int32_t)-1;
      }
      if (flags & kEpDone) L.tfz[t] |= 2u;  // held from the next step on
    }
    st[kEpFlags] = flags;
  }
}

// wave-uniform phase timer: adds the cycles since the previous mark to counter k
struct PhaseTimer {
  unsigned long long last;
  __device__ __forceinline__ void mark(const Lds& L, int lane, int k) {
    const unsigned long long t = (unsigned long long)clock64();
    if (lane == 0) L.cyc[k] += t - last;
    last = t;
  }
};

__device__ __forceinline__ uint64_t lane_lt_mask(int lane) { return lane ? ((~0ull) >> (64 - lane)) : 0ull; }

// SAT on up to 64 ring entries starting at `head`; colliding pairs are appended (in order)
// to the canonical list, a box pair's normal and depth beside it (msat), for its manifold.
// Returns the new list length.
__device__ __forceinline__ int narrow_chunk(const Lds& L, int head, int count, int nman, int lane) {
  const int NB = L.nbp;
  bool hit = false, ground = true;
  uint32_t code = 0;
  float n[3] = {0.f, 0.f, 0.f}, depth = 0.f;
  if (lane < count) {
    code = L.ring[(head + lane) & (kRing - 1)];
    const int i = (int)(code >> 16), j = (int)(code & 0xffffu);
    ground = j == (int)kGround;
    if (ground) {
      hit = L.x[2 * NB + i] - L.hm[2 * NB + i] < 0.f;
    } else {
      float RA[9], RB[9], heA[3], heB[3], d[3];
      body_R(L, i, RA);
      body_R(L, j, RB);
      load3(L.he, NB, i, heA);
      load3(L.he, NB, j, heB);
#pragma unroll
      for (int k = 0; k < 3; ++k) d[k] = L.x[k * NB + j] - L.x[k * NB + i];
      hit = sat_boxes(RA, heA, RB, heB, d, n, depth);
    }
  }
  const uint64_t bal = __ballot(hit);
  if (hit) {
    const int idx = nman + __popcll(bal & lane_lt_mask(lane));
    if (idx < L.pc) {
      L.cab[idx] = code;
      if (!ground) *reinterpret_cast<float4*>(L.msat + 4 * (size_t)idx) = make_float4(n[0], n[1], n[2], depth);
    }
  }
  return nman + __popcll(bal);
}

// ------------------------------------------------------------------------------------------------
// the kernel
// ------------------------------------------------------------------------------------------------
// kLearned: the variant with contact features (learned warm start, feature records); the plain
// variant does not carry the network's registers.
// kGlobal: the pack's layout lives in its region of device memory instead of LDS.  The two are
// separate instantiations so that the LDS variant's accesses compile to LDS instructions.
// A device-memory variant runs several waves: the first runs every phase, and the others join
// it where an island's work is wide (the broadphase walk, the manifolds, the sweeps, the residual
// terms).  The plain variant runs kIslandWaves waves; the one with the network's registers (one
// wave per SIMD) runs four, one per SIMD of the compute unit.
template <bool kLearned, bool kGlobal, bool kLat = false>
constexpr int step_threads() {
  return kGlobal ? (kLearned ? kLearnedIslandWaves : kIslandWaves) * kWave : (kLat ? kLatencyWaves * kWave : kWave);
}

// The plain variants are held to two waves per SIMD (at most 256 registers): occupancy is what
// hides the latency of the pack's serial phases, and a register count that drifts above 256
// would halve it.
// kHot (packs in device memory): the body arrays of the serial walks are in LDS too.  It is a
// template parameter so that every access has one known address space (a pointer that may be
// either compiles to flat instructions, which are as slow as device memory even on LDS).
// kExt: the solver variants (disc friction, restitution targets, reference-face clipping) and the
// episode criteria are compiled in; the default plain kernel carries none of their registers.
// kLat (small batches): one tower per workgroup of kLatencyWaves waves; the first wave steps it as
// a pack, the others join it in building the manifolds, in the sweeps (register-resident lane
// pairs, pgs_sweeps_lat) and in the residual terms.
template <bool kLearned, bool kGlobal, bool kHot, bool kExt, bool kLat = false>
__global__ void __launch_bounds__((step_threads<kLearned, kGlobal, kLat>()))
__attribute__((amdgpu_waves_per_eu(kLearned ? 1 : 2))) step_kernel(StepArgs a) {
  constexpr int kThreads = step_threads<kLearned, kGlobal, kLat>();
  extern __shared__ __align__(16) float smem[];
  float* const dev = a.gmem + a.pack_goff[a.pack_first + blockIdx.x];
  const Lds L = carve(kGlobal ? dev + kManPackWords * a.pc : smem, dev, smem, kGlobal, kGlobal && kHot, a);
  const bool keep_prev = lds_mode(a) >= 1;   // previous-step store kept (warm start or records)
  if constexpr (kThreads > kWave) {
    if (threadIdx.x >= kWave) {
      // helper waves: per substep they join the first wave in the broadphase walk (islands in
      // device memory), in building the manifolds, in the sweeps and in the residual terms, each
      // between a barrier where it enters and one where it leaves (the same barriers, in the
      // same order, as the first wave's) (with the learned warm start they share the network's
      // chunks too; the sweeps after it are mlp_iters, and its own residual and fallback stay
      // with the first wave)
      const int pkh = a.pack_first + blockIdx.x;
      const int nbh = a.pack_body0[pkh + 1] - a.pack_body0[pkh];
      const bool learned_h = kLearned && a.warm_start == 2;
      const int slot0h = a.pack_slot0[pkh];
      const float gdt_h = sqrtf(a.g[0] * a.g[0] + a.g[1] * a.g[1] + a.g[2] * a.g[2]) * a.dt;
      const SolveOpts opts_h = {a.restitution, kExt && a.friction_cone != 0, kExt && a.restitution_bias != 0};
      for (int s = 0; s < a.n_steps; ++s)
        for (int sub = 0; sub < a.n_sub; ++sub) {
          if constexpr (kGlobal) {
            __syncthreads();
            island_walk_rounds(L, a.margin, nbh, threadIdx.x / kWave, kThreads / kWave, threadIdx.x % kWave);
            __syncthreads();
          }
          __syncthreads();
          build_manifolds<kExt>(L, a, threadIdx.x, kThreads, L.scal[5], keep_prev);
          __syncthreads();
          if constexpr (kLearned) {
            const bool rec_h = a.feat_out != nullptr && s == a.n_steps - 1 && sub == a.n_sub - 1;
            if (learned_h || rec_h) {
              const int wv = threadIdx.x / kWave;
              __syncthreads();
              learned_chunks(L, a, L.coloff[L.scal[2]], slot0h, gdt_h, learned_h, rec_h, wv, kThreads / kWave,
                             threadIdx.x % kWave, L.xs ? L.xs + wv * kStageWords : nullptr);
              __syncthreads();
            }
          }
          __syncthreads();
          if constexpr (kLat) pgs_sweeps_lat<kThreads>(L, a.iters, L.scal[2], threadIdx.x, opts_h);
          else pgs_sweeps(L, learned_h ? a.mlp_iters : a.iters, L.scal[2], threadIdx.x, kThreads, opts_h);
          __syncthreads();
          if (!learned_h && s == a.n_steps - 1 && sub == a.n_sub - 1) {
            __syncthreads();
            residual_parts(L, L.scal[5], threadIdx.x, kThreads, reinterpret_cast<float*>(L.cab),
                           reinterpret_cast<float*>(L.cpos), nullptr, opts_h);
            __syncthreads();
          }
        }
      return;
    }
  }
  const int lane = threadIdx.x;
  const int pk = a.pack_first + blockIdx.x;
  const int gb0 = a.pack_body0[pk], nb = a.pack_body0[pk + 1] - gb0;
  const int gt0 = a.pack_tower0[pk], nt = a.pack_tower0[pk + 1] - gt0;
  const int gp0 = a.pack_push0[pk], np = a.pack_push0[pk + 1] - gp0;
  const int slot0 = a.pack_slot0[pk];
  const int NB = L.nbp, PC = L.pc, CAP = a.cap;
  PhaseTimer timer;
  timer.last = (unsigned long long)clock64();
  if (lane < kPhases) L.cyc[lane] = 0ull;

  // ---- load the pack ----
  for (int i = lane; i < nb; i += kWave) {
    const int g = gb0 + i;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      L.x[k * NB + i] = a.x[k * CAP + g];
      L.v[k * NB + i] = a.v[k * CAP + g];
      L.w[k * NB + i] = a.w[k * CAP + g];
      L.he[k * NB + i] = a.he[k * CAP + g];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) L.q[k * NB + i] = a.q[k * CAP + g];
    // inverse mass (the inverse body inertia is taken from the mass and the sizes where needed)
    const float m = a.mass[g];
    const bool dyn = m > 0.f;
    L.invm[i] = dyn ? 1.f / m : 0.f;
    L.flag[i] = a.flags[g];
    L.tw[i] = a.body_tower[g] - gt0;
    if (!dyn) {
#pragma unroll
      for (int k = 0; k < 3; ++k) { L.v[k * NB + i] = 0.f; L.w[k * NB + i] = 0.f; }
    }
  }
  for (int t = lane; t < nt; t += kWave) {
    L.tb0[t] = a.tower_body0[gt0 + t] - gb0;
    L.tb1[t] = a.tower_body0[gt0 + t + 1] - gb0;
    L.mu[t] = a.tower_mu[gt0 + t];
    // bit 1: non-finite state (held); bit 2: episode done (held); bit 4: collapse declared
    uint32_t fz = a.tower_frozen[gt0 + t] ? 1u : 0u;
    if (kExt && a.ep_state) {
      const uint32_t ef = a.ep_state[(size_t)(gt0 + t) * kEpisodeWords + kEpFlags];
      fz |= ((ef & kEpDone) ? 2u : 0u) | ((ef & kEpCollapsed) ? 4u : 0u);
    }
    L.tfz[t] = fz;
#pragma unroll
    for (int k = 0; k < 4; ++k) L.tcnt[t * 4 + k] = 0u;
    L.tres[2 * t] = 0.f;
    L.tres[2 * t + 1] = 0.f;
  }
  for (int r = lane; r < np; r += kWave) {
    const int g = gp0 + r;
    L.pb[r] = a.push_body[g] - gb0;
    L.ps[r] = a.push_start[g];
    L.pn[r] = a.push_steps[g];
#pragma unroll
    for (int k = 0; k < 3; ++k) { L.pf[3 * r + k] = a.push_force[3 * g + k]; L.px0[3 * r + k] = a.push_x0[3 * g + k]; }
    L.pwd[r] = a.push_withdraw[g];
  }
  if (lane == 0) {
    L.scal[3] = 0;                                   // error bits
    // an on-chip pack holds at most kWindows x 64 bodies (the host sizes them so)
    if (!kGlobal && nb > kWindows * kWave) L.scal[3] = kErrCand;
    L.scal[4] = keep_prev ? a.prev_count[pk] : 0;    // previous-step manifolds
  }
  if constexpr (kLearned) {
    if (a.warm_start == 2)
      for (int t = lane; t < nt; t += kWave) { L.tfc[2 * t] = 0u; L.tfc[2 * t + 1] = 0u; }
  }
  if (keep_prev) {
    const int npv = a.prev_count[pk];
    for (int p = lane; p < npv; p += kWave) {
      const int g = slot0 + p;
      L.pkey[p] = a.prev_key[g];
      L.pslot[p] = __float_as_uint(a.prev_data[16 * g + 3]);
#pragma unroll
      for (int k = 0; k < 3; ++k) L.pnrm[k * PC + p] = a.prev_data[16 * g + k];
#pragma unroll
      for (int k = 0; k < 12; ++k) L.plam[k * PC + p] = a.prev_data[16 * g + 4 + k];
    }
  }
  wave_sync();
  // a tower with a non-finite body (state set by the host) is frozen from the first step on
  for (int i = lane; i < nb; i += kWave) {
    if (!(L.flag[i] & kActive)) continue;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      finite = finite && isfinite(L.x[k * NB + i]) && isfinite(L.v[k * NB + i]) && isfinite(L.w[k * NB + i]);
#pragma unroll
    for (int k = 0; k < 4; ++k) finite = finite && isfinite(L.q[k * NB + i]);
    if (!finite) {
      atomicOr(&L.tfz[L.tw[i]], 1u);
      atomicOr((uint32_t*)&L.scal[3], kErrNan);
    }
  }
  wave_sync();
  timer.mark(L, lane, 0);

  const float dt = a.dt, e = a.restitution;
  const SolveOpts opts = {e, kExt && a.friction_cone != 0, kExt && a.restitution_bias != 0};
  for (int s = 0; s < a.n_steps; ++s) {
    const int64_t step = a.step0 + s;
    for (int r = lane; r < np; r += kWave)
      if ((int64_t)L.ps[r] == step) {
        const int b = L.pb[r];
#pragma unroll
        for (int k = 0; k < 3; ++k) L.px0[3 * r + k] = L.x[k * NB + b];
      }
    wave_sync();
    for (int sub = 0; sub < a.n_sub; ++sub) {
      const bool last = (s == a.n_steps - 1) && (sub == a.n_sub - 1);
      // ---- the bodies of a frozen tower (non-finite state, found at the launch's start or by
      // the integration) or of an episode at rest are held: they neither move nor collide and keep
      // their state ----
      for (int i = lane; i < nb; i += kWave) {
        const uint32_t f = L.flag[i];
        if ((f & kActive) && (L.tfz[L.tw[i]] & 3u)) L.flag[i] = (f & ~kActive) | kHeld;
      }
      wave_sync();
      // ---- 1. external forces; 2. frames ----
      for (int i = lane; i < nb; i += kWave) {
        const uint32_t f = L.flag[i];
        const bool moving = (f & (kActive | kDynamic)) == (kActive | kDynamic);
        if (moving) {
          float vv[3];
          load3(L.v, NB, i, vv);
#pragma unroll
          for (int k = 0; k < 3; ++k) vv[k] += dt * a.g[k];
          const float im = L.invm[i];
          const bool pushes_on = !(L.tfz[L.tw[i]] & 4u);   // none after a declared collapse
          for (int r = 0; r < np; ++r)
            if (pushes_on && L.pb[r] == i && step >= (int64_t)L.ps[r] && step < (int64_t)L.ps[r] + L.pn[r]) {
#pragma unroll
              for (int k = 0; k < 3; ++k) vv[k] += dt * L.pf[3 * r + k] * im;
            }
          store3(L.v, NB, i, vv);
        }
        float R[9];
        body_R(L, i, R);
        const float he0 = L.he[i], he1 = L.he[NB + i], he2 = L.he[2 * NB + i];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          L.hm[k * NB + i] = fabsf(R[3 * k]) * he0 + fabsf(R[3 * k + 1]) * he1 + fabsf(R[3 * k + 2]) * he2;
        float d[3];
        if (moving) inv_body_inertia(L, i, a.mass[gb0 + i], d);
        else d[0] = d[1] = d[2] = 0.f;
        // R diag(d) R^T
        L.Iw[i] = R[0] * d[0] * R[0] + R[1] * d[1] * R[1] + R[2] * d[2] * R[2];
        L.Iw[NB + i] = R[3] * d[0] * R[3] + R[4] * d[1] * R[4] + R[5] * d[2] * R[5];
        L.Iw[2 * NB + i] = R[6] * d[0] * R[6] + R[7] * d[1] * R[7] + R[8] * d[2] * R[8];
        L.Iw[3 * NB + i] = R[0] * d[0] * R[3] + R[1] * d[1] * R[4] + R[2] * d[2] * R[5];
        L.Iw[4 * NB + i] = R[0] * d[0] * R[6] + R[1] * d[1] * R[7] + R[2] * d[2] * R[8];
        L.Iw[5 * NB + i] = R[3] * d[0] * R[6] + R[4] * d[1] * R[7] + R[5] * d[2] * R[8];
      }
      for (int c = lane; c <= kMaxColours; c += kWave) L.colcnt[c] = 0;
      for (int t = lane; t < nt; t += kWave) {
        L.tcnt[t * 4 + 3] = 0u;
        L.tc0[t] = 0;
        L.tc1[t] = 0;
        L.tpts[t] = 0;
      }
      wave_sync();
      timer.mark(L, lane, 1);

      // ---- 3 + 4. broadphase in canonical order, narrowphase on every 64 candidates ----
      // Lane l holds body 64 w + l of window w in registers (position, AABB, flags, tower);
      // body i is broadcast from its window with readlane, so the pair loop touches LDS only
      // to append candidates to the ring.
      int head = 0, tail = 0, nman = 0;
      if constexpr (kGlobal) {
        // islands in device memory (one tower each).  Bounding boxes of 64-body windows filter
        // the pair tests; each lane then walks its own body's candidates j > i in ascending
        // order, the ground last, into that body's own slots.  A scan of the counts gives each
        // body its place in the canonical list, the runs are copied there, and the SAT runs on
        // that list 64 at a time, so the candidates keep their canonical order.
        const int nwin = (nb + kWave - 1) / kWave;
        for (int w = lane; w < nwin; w += kWave) {
          float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
          for (int j = w * kWave; j < min(nb, (w + 1) * kWave); ++j) {
            if (!(L.flag[j] & kActive)) continue;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              lo[k] = fminf(lo[k], L.x[k * NB + j] - L.hm[k * NB + j]);
              hi[k] = fmaxf(hi[k], L.x[k * NB + j] + L.hm[k * NB + j]);
            }
          }
#pragma unroll
          for (int k = 0; k < 3; ++k) { L.wbox[6 * w + k] = lo[k]; L.wbox[6 * w + 3 + k] = hi[k]; }
        }
        wave_sync();
        // one walk: each body's candidates into its own kCandPerBody slots, counts into the (still
        // unused) colouring lane masks; an exclusive scan of the counts places each body's run in
        // the canonical list, and the runs are copied there.  A body with more candidates than
        // its slots keeps the first kCandPerBody (flagged).  The helper waves share the walk.
        uint32_t* const cnt = L.lmlo;
        if constexpr (kThreads > kWave) {
          __syncthreads();   // window boxes, frames and flags are in place; the helpers enter
          island_walk_rounds(L, a.margin, nb, 0, kThreads / kWave, lane);
          __syncthreads();   // every body's candidates are in its slots
        } else {
          island_walk_rounds(L, a.margin, nb, 0, 1, lane);
          wave_sync();
        }
        uint32_t run = 0;
        for (int i0 = 0; i0 < nb; i0 += kWave) {
          const int i = i0 + lane;
          const uint32_t c = i < nb ? cnt[i] : 0u;
          uint32_t incl = c;
#pragma unroll
          for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t t = __shfl_up(incl, d);
            if (lane >= d) incl += t;
          }
          if (i < nb) {
            const uint32_t off = run + incl - c;
            uint32_t v[kCandPerBody];
#pragma unroll
            for (int k = 0; k < kCandPerBody; ++k)
              if (k < (int)c) v[k] = L.cslot[i * kCandPerBody + k];
#pragma unroll
            for (int k = 0; k < kCandPerBody; ++k)
              if (k < (int)c) L.cand[off + k] = v[k];
          }
          run += __shfl(incl, kWave - 1);
        }
        const int total = (int)run;
        wave_sync();
        for (int c0 = 0; c0 < total; c0 += kWave) {
          const int n = min(kWave, total - c0);
          // narrow_chunk reads the ring: stage the next 64 candidates there
          if (lane < n) L.ring[(head + lane) & (kRing - 1)] = L.cand[c0 + lane];
          wave_sync();
          nman = narrow_chunk(L, head, n, nman, lane);
          head += n;
          wave_sync();
        }
        tail = head;
        if (lane == 0) L.tcnt[0] += (uint32_t)run;   // an island is one tower (kept candidates)
      } else {
        float wx[kWindows][3], wh[kWindows][3];
        uint32_t wf[kWindows];
        int wt[kWindows];
#pragma unroll
        for (int w = 0; w < kWindows; ++w) {
          const int j = w * kWave + lane;
          const bool in = j < nb;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            wx[w][k] = in ? L.x[k * NB + j] : 0.f;
            wh[w][k] = in ? L.hm[k * NB + j] : 0.f;
          }
          wf[w] = in ? L.flag[j] : 0u;
          wt[w] = in ? L.tw[j] : -1;
        }
        const int nwin = (nb + kWave - 1) / kWave;
        int cur_t = -1, cand_acc = 0;
        for (int i = 0; i < nb; ++i) {
          const int wi = i / kWave, li = i % kWave;
          float xi[3], hi[3];
          uint32_t fi = 0u;
          int ti = 0;
#pragma unroll
          for (int w = 0; w < kWindows; ++w)
            if (w == wi) {
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                xi[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wx[w][k]), li));
                hi[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wh[w][k]), li));
              }
              fi = __builtin_amdgcn_readlane(wf[w], li);
              ti = __builtin_amdgcn_readlane(wt[w], li);
            }
          if (!(fi & kActive)) continue;
          if (ti != cur_t) {
            if (lane == 0 && cur_t >= 0 && cand_acc) L.tcnt[cur_t * 4 + 0] += (uint32_t)cand_acc;
            cur_t = ti;
            cand_acc = 0;
          }
          const bool dyni = (fi & kDynamic) != 0;
#pragma unroll
          for (int w = 0; w < kWindows; ++w) {
            if (w < wi || w >= nwin) continue;
            const int j = w * kWave + lane;
            const bool hit = j > i && wt[w] == ti && (wf[w] & kActive) && (dyni || (wf[w] & kDynamic)) &&
                             fabsf(xi[0] - wx[w][0]) <= hi[0] + wh[w][0] + a.margin &&
                             fabsf(xi[1] - wx[w][1]) <= hi[1] + wh[w][1] + a.margin &&
                             fabsf(xi[2] - wx[w][2]) <= hi[2] + wh[w][2] + a.margin;
            const uint64_t bal = __ballot(hit);
            if (hit) L.ring[(tail + __popcll(bal & lane_lt_mask(lane))) & (kRing - 1)] = ((uint32_t)i << 16) | (uint32_t)j;
            const int cnt = __popcll(bal);
            cand_acc += cnt;
            tail += cnt;
            if (tail - head >= kWave) {
              wave_sync();
              nman = narrow_chunk(L, head, kWave, nman, lane);
              head += kWave;
            }
          }
          // the ground comes last in body i's canonical row
          if (dyni && (xi[2] - hi[2] <= a.margin)) {
            if (lane == 0) L.ring[tail & (kRing - 1)] = ((uint32_t)i << 16) | kGround;
            cand_acc += 1;
            tail += 1;
            if (tail - head >= kWave) {
              wave_sync();
              nman = narrow_chunk(L, head, kWave, nman, lane);
              head += kWave;
            }
          }
        }
        if (lane == 0 && cur_t >= 0 && cand_acc) L.tcnt[cur_t * 4 + 0] += (uint32_t)cand_acc;
      }
      wave_sync();
      while (head < tail) {
        const int cnt = min(kWave, tail - head);
        nman = narrow_chunk(L, head, cnt, nman, lane);
        head += cnt;
      }
      if (nman > PC) {
        if (lane == 0) L.scal[3] |= kErrMan;
        nman = PC;
      }
      wave_sync();
      timer.mark(L, lane, 2);

      // ---- 5. tower ranges of the canonical list; greedy first-fit colouring ----
      if (nt == 1) {
        if (lane == 0 && nman > 0) { L.tc0[0] = 0; L.tc1[0] = nman; }
      } else {
        for (int p = lane; p < nman; p += kWave) {
          const int t = L.tw[L.cab[p] >> 16];
          if (p == 0 || L.tw[L.cab[p - 1] >> 16] != t) L.tc0[t] = p;
          if (p == nman - 1 || L.tw[L.cab[p + 1] >> 16] != t) L.tc1[t] = p + 1;
        }
      }
      // per-body lane masks of the current chunk (the sorted-manifold words are free until the
      // manifolds are written): lanes that touch body i, low and high 32 lanes
      uint32_t* const lmlo = L.lmlo;
      uint32_t* const lmhi = L.lmhi;
      for (int i = lane; i < nb; i += kWave) { L.hm[i] = 0.f; L.hm[NB + i] = 0.f; lmlo[i] = 0u; lmhi[i] = 0u; }
      wave_sync();
      uint32_t* mask = (uint32_t*)L.hm;   // [word * nbp + body]
      // Greedy first fit in canonical order, 64 manifolds at a time: a lane is coloured once
      // every earlier manifold of its chunk that shares a dynamic body is coloured.  Lanes
      // coloured in one round share no body, and each sees exactly the colours of all its
      // earlier neighbours, so the result equals the sequential greedy colouring.
      // (the next chunk's codes are loaded while this one is coloured)
      uint32_t code_next = lane < nman ? L.cab[lane] : 0u;
      for (int c0 = 0; c0 < nman; c0 += kWave) {
        const int p = c0 + lane;
        const bool valid = p < nman;
        const uint32_t code = code_next;
        code_next = p + kWave < nman ? L.cab[p + kWave] : 0u;
        const int i = (int)(code >> 16), j = (int)(code & 0xffffu);
        const bool di = valid && (L.flag[i] & kDynamic);
        const bool dj = valid && j != (int)kGround && (L.flag[j] & kDynamic);
        // earlier lanes of the chunk that share a dynamic body with this one
        uint32_t* const lmw = lane < 32 ? lmlo : lmhi;
        const uint32_t lbit = 1u << (lane & 31);
        if (di) atomicOr(&lmw[i], lbit);
        if (dj) atomicOr(&lmw[j], lbit);
        wave_sync();
        uint64_t dep = 0ull;
        if (di) dep |= ((uint64_t)lmhi[i] << 32) | lmlo[i];
        if (dj) dep |= ((uint64_t)lmhi[j] << 32) | lmlo[j];
        dep &= lane_lt_mask(lane);
        wave_sync();
        if (di) { lmlo[i] = 0u; lmhi[i] = 0u; }
        if (dj) { lmlo[j] = 0u; lmhi[j] = 0u; }
        bool done = !valid;
        int col = -1;
        if constexpr (kGlobal) {
          // An island's chunks take many rounds (its canonical order runs along chains of
          // touching stones), so the rounds stay in registers: the colours a lane may not take
          // are those its bodies got in earlier chunks (read once) and those of the earlier lanes
          // of this chunk it depends on, folded in (by broadcast) in the round after each is
          // coloured; the chunk's colours go into the body masks at its end.
          uint64_t u = 0ull;
          if (di) u |= (uint64_t)mask[i] | ((uint64_t)mask[NB + i] << 32);
          if (dj) u |= (uint64_t)mask[j] | ((uint64_t)mask[NB + j] << 32);
          uint64_t fresh = 0ull;   // lanes coloured in the previous round (wave-uniform)
          while (true) {
            for (uint64_t f = fresh; f != 0ull; f &= f - 1ull) {
              const int k = __ffsll((unsigned long long)f) - 1;
              const int ck = __builtin_amdgcn_readlane(col, k);
              if (ck >= 0 && ((dep >> k) & 1ull)) u |= 1ull << ck;
            }
            const uint64_t donem = __ballot(done);
            if (donem == ~0ull) break;
            const bool ready = !done && (dep & ~donem) == 0ull;
            if (ready) {
              if (u != ~0ull) col = __ffsll((unsigned long long)~u) - 1;
              done = true;
            }
            fresh = __ballot(ready);
          }
          // lanes that share a body set different bits
          if (valid && col >= 0) {
            const uint64_t bit = 1ull << col;
            if (di) { atomicOr(&mask[i], (uint32_t)bit); atomicOr(&mask[NB + i], (uint32_t)(bit >> 32)); }
            if (dj) { atomicOr(&mask[j], (uint32_t)bit); atomicOr(&mask[NB + j], (uint32_t)(bit >> 32)); }
          }
          wave_sync();   // the masks are complete before the next chunk reads them
        } else {
          // a pack's chunks take few rounds, each colouring many lanes: the masks stay in LDS
          while (true) {
            const uint64_t donem = __ballot(done);
            if (donem == ~0ull) break;
            if (!done && (dep & ~donem) == 0ull) {
              uint64_t u = 0ull;
              if (di) u |= (uint64_t)mask[i] | ((uint64_t)mask[NB + i] << 32);
              if (dj) u |= (uint64_t)mask[j] | ((uint64_t)mask[NB + j] << 32);
              if (u != ~0ull) {
                col = __ffsll((unsigned long long)~u) - 1;
                const uint64_t bit = 1ull << col;
                if (di) { mask[i] |= (uint32_t)bit; mask[NB + i] |= (uint32_t)(bit >> 32); }
                if (dj) { mask[j] |= (uint32_t)bit; mask[NB + j] |= (uint32_t)(bit >> 32); }
              }
              done = true;
            }
            wave_sync();
          }
        }
        if (valid) {
          L.cpos[p] = col;
          if (col >= 0) atomicAdd(&L.colcnt[col], 1);
          else atomicOr((uint32_t*)&L.scal[3], kErrCol);
        }
      }
      wave_sync();
      // colour offsets (wave prefix sum over the 64 colour counts)
      {
        const int cnt = L.colcnt[lane];
        int incl = cnt;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
          const int t = __shfl_up(incl, d);
          if (lane >= d) incl += t;
        }
        L.coloff[lane + 1] = incl;
        L.colcnt[lane] = incl - cnt;       // running position of each colour
        if (lane == 0) L.coloff[0] = 0;
        const uint64_t used = __ballot(cnt > 0);
        if (lane == 0) L.scal[2] = used ? 64 - __clzll((long long)used) : 0;
      }
      wave_sync();
      // colour-sorted positions, canonical order inside each colour
      int col_next = lane < nman ? L.cpos[lane] : -1;
      for (int c0 = 0; c0 < nman; c0 += kWave) {
        const int p = c0 + lane;
        const int col = col_next;
        col_next = p + kWave < nman ? L.cpos[p + kWave] : -1;
        int pos = -1;
        uint64_t pending = __ballot(col >= 0);
        while (pending) {
          const int c = __builtin_amdgcn_readlane(col, __ffsll((unsigned long long)pending) - 1);
          const uint64_t m = __ballot(col == c);
          const int base = L.colcnt[c];
          if (col == c) pos = base + __popcll(m & lane_lt_mask(lane));
          wave_sync();
          if (lane == 0) L.colcnt[c] = base + __popcll(m);
          wave_sync();
          pending &= ~m;
        }
        if (p < nman) {
          L.cpos[p] = pos;
          if (col >= 0) atomicMax(&L.tcnt[(nt == 1 ? 0 : L.tw[L.cab[p] >> 16]) * 4 + 3], (uint32_t)(col + 1));
        }
      }
      wave_sync();
      timer.mark(L, lane, 3);
      const int ncol = L.scal[2];
      const int nkept = L.coloff[ncol];

      // ---- 6. manifolds into colour-sorted slots (+ warm start lookup) ----
      // (an island's helper waves join in between the two barriers)
      if constexpr (kThreads > kWave) {
        L.scal[5] = nman;
        __syncthreads();
        build_manifolds<kExt>(L, a, threadIdx.x, kThreads, nman, keep_prev);
        __syncthreads();
      } else {
        build_manifolds<kExt>(L, a, lane, kWave, nman, keep_prev);
        wave_sync();
      }
      timer.mark(L, lane, 4);

      // ---- learned warm start: features, network, initial impulses; feature records ----
      bool learned = false;
      if constexpr (kLearned) {
        learned = a.warm_start == 2;
        const bool rec = a.feat_out != nullptr && last;
        if (learned)
          for (int i = lane; i < nb; i += kWave)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              L.vsave[k * NB + i] = L.v[k * NB + i];
              L.vsave[(3 + k) * NB + i] = L.w[k * NB + i];
            }
        if (learned || rec) {
          const float gdt = sqrtf(a.g[0] * a.g[0] + a.g[1] * a.g[1] + a.g[2] * a.g[2]) * dt;
          if constexpr (kThreads > kWave) {
            // an island's helper waves take chunks too, each with its own staging rows
            __syncthreads();
            learned_chunks(L, a, nkept, slot0, gdt, learned, rec, 0, kThreads / kWave, lane, L.xs);
            __syncthreads();
          } else {
            learned_chunks(L, a, nkept, slot0, gdt, learned, rec, 0, 1, lane, L.xs);
          }
          wave_sync();
        }
        if (keep_prev && a.warm_start == 0) {
          // records without a warm start: the key lookup filled ml only to feed the features
          // (on every step, so the solve starts from zero whether or not this step records)
          for (int m = lane; m < nkept; m += kWave)
#pragma unroll
            for (int k = 0; k < 12; ++k) mdev(L, m)[12 + k] = 0.f;
          wave_sync();
        }
      }

      // ---- 7. warm-start impulses, then PGS sweeps, colour by colour ----
      if (a.warm_start == 1) {
        for (int col = 0; col < ncol; ++col) {
          for (int m = L.coloff[col] + lane; m < L.coloff[col + 1]; m += kWave) warm_apply_manifold(L, m);
          wave_sync();
        }
      }
      int sweeps = a.iters;
      if constexpr (kLearned) {
        if (learned) {
          const float gdt = sqrtf(a.g[0] * a.g[0] + a.g[1] * a.g[1] + a.g[2] * a.g[2]) * dt;
          for (int col = 0; col < ncol; ++col) {
            for (int m = L.coloff[col] + lane; m < L.coloff[col + 1]; m += kWave)
              learned_apply_manifold(L, m, L.mu[L.tw[L.mab[m] >> 16]], gdt, opts.cone);
            wave_sync();
          }
          sweeps = a.mlp_iters;
        }
      }
      __syncthreads();   // the helper waves (if any) enter the sweeps with this wave
      if constexpr (kLat) pgs_sweeps_lat<kThreads>(L, sweeps, ncol, threadIdx.x, opts);
      else pgs_sweeps(L, sweeps, ncol, threadIdx.x, kThreads, opts);
      __syncthreads();
      timer.mark(L, lane, 5);

      // ---- learned warm start: residual, and the plain solve again for towers above tau ----
      if constexpr (kLearned) {
        if (learned) {
          tower_residuals(L, nman, nt, lane, L.rpart, L.rpart + PC, nullptr, opts);
          wave_sync();
          int any = 0;
          for (int t = lane; t < nt; t += kWave) {
            const uint32_t fb = L.tres[2 * t] > a.fallback_tau ? 1u : 0u;
            L.tfb[t] = fb;
            any |= (int)fb;
          }
          wave_sync();
          any = __any(any);   // one wave per workgroup: a wave vote is the workgroup's
          if (any) {
            for (int i = lane; i < nb; i += kWave)
              if (L.tfb[L.tw[i]])
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                  L.v[k * NB + i] = L.vsave[k * NB + i];
                  L.w[k * NB + i] = L.vsave[(3 + k) * NB + i];
                }
            for (int m = lane; m < nkept; m += kWave)
              if (L.tfb[L.tw[L.mab[m] >> 16]])
#pragma unroll
                for (int k = 0; k < 12; ++k) mdev(L, m)[12 + k] = 0.f;
            wave_sync();
            for (int it = 0; it < a.iters; ++it) {
              for (int col = 0; col < ncol; ++col) {
                for (int m = L.coloff[col] + lane; m < L.coloff[col + 1]; m += kWave) {
                  const int t = L.tw[L.mab[m] >> 16];
                  if (L.tfb[t]) solve_manifold(L, m, opts);
                }
                wave_sync();
              }
            }
            for (int t = lane; t < nt; t += kWave)
              if (L.tfb[t]) { L.tfc[2 * t] += 1u; L.tfc[2 * t + 1] += (uint32_t)L.tpts[t]; }
            tower_residuals(L, nman, nt, lane, L.rpart, L.rpart + PC, L.tfb, opts);
          }
          wave_sync();
          timer.mark(L, lane, 7);
        }
      }

      // ---- contacts of the final step; warm-start store ----
      if (last) {
        for (int m = lane; m < nkept; m += kWave) {
          int col = 0;
          while (col + 1 < ncol && L.coloff[col + 1] <= m) ++col;
          const int a_ = (int)(L.mab[m] >> 16);
          const int g = slot0 + m;
          a.out_ab[g] = L.mab[m];
          a.out_meta[g] = (L.mmeta[m] & 0x0ffff00fu) | ((uint32_t)col << 4);
          a.out_tower[g] = L.tw[a_];
          const float nn[3] = {mdev(L, m)[24], mdev(L, m)[25], mdev(L, m)[26]};
          Frame F;
          make_frame(nn, F);
          for (int k = 0; k < 3; ++k) {
            a.out_geo[8 * g + k] = nn[k];
            a.out_geo[8 * g + 3 + k] = F.f[1][k];
          }
          a.out_geo[8 * g + 6] = mdev(L, m)[27];
          a.out_geo[8 * g + 7] = 0.f;
          const int npts = (int)(L.mmeta[m] & 15u);
          if constexpr (kLearned) {
            if (a.feat_out) record_solution(L, m, a.feat_out + (size_t)g * 4 * kFeatRecord);
          }
          for (int q = 0; q < 4; ++q) {
            float rl[3] = {0.f, 0.f, 0.f}, rw[3];
            if (q < npts)
              for (int k = 0; k < 3; ++k) rl[k] = mdev(L, m)[q * 3 + k];
            to_world(F, rl, rw);
            for (int k = 0; k < 3; ++k) {
              a.out_pts[24 * g + 6 * q + k] = L.x[k * NB + a_] + rw[k];
              a.out_pts[24 * g + 6 * q + 3 + k] = q < npts ? mdev(L, m)[12 + q * 3 + k] : 0.f;
            }
          }
        }
        if (lane == 0) a.out_count[pk] = nkept;
      }
      if (keep_prev) {
        // canonical-order store of this step's impulses (dropped pairs keep their key, no points)
        for (int p = lane; p < nman; p += kWave) { L.pkey[p] = L.cab[p]; L.pslot[p] = 0u; }
        wave_sync();
        for (int m = lane; m < nkept; m += kWave) {
          const int p = L.mcanon[m];
          const uint32_t meta = L.mmeta[m];
          const int npts = (int)(meta & 15u);
          L.pslot[p] = (uint32_t)npts | (((meta >> 12) & 0xffffu) << 4);
#pragma unroll
          for (int k = 0; k < 3; ++k) L.pnrm[k * PC + p] = mdev(L, m)[24 + k];
          for (int k = 0; k < 12; ++k) L.plam[k * PC + p] = mdev(L, m)[12 + k];
        }
        if (lane == 0) L.scal[4] = nman;
      }
      wave_sync();
      timer.mark(L, lane, 6);

      // ---- 8. residual of the launch's last solve, the one the outputs report (the learned
      // variant took it before the outputs, for its fallback) ----
      if (!learned && last) {
        float* const psum = reinterpret_cast<float*>(L.cab);
        float* const pmax = reinterpret_cast<float*>(L.cpos);
        if constexpr (kThreads > kWave) {
          // an island's helper waves join in the pairs' terms
          __syncthreads();
          residual_parts(L, nman, threadIdx.x, kThreads, psum, pmax, nullptr, opts);
          __syncthreads();
          tower_residuals(L, nman, nt, lane, psum, pmax, nullptr, opts, false);
        } else {
          tower_residuals(L, nman, nt, lane, psum, pmax, nullptr, opts);
        }
        timer.mark(L, lane, 7);
      }

      // ---- 9. integrate ----
      for (int i = lane; i < nb; i += kWave) {
        const uint32_t f = L.flag[i];
        if ((f & (kActive | kDynamic)) != (kActive | kDynamic)) continue;
        if (!integrate_body(L, i, a.mass[gb0 + i], dt)) {
          atomicOr((uint32_t*)&L.scal[3], kErrNan);
          atomicOr(&L.tfz[L.tw[i]], 1u);   // frozen from the next substep on
        }
      }
      wave_sync();
      timer.mark(L, lane, 8);
      // ---- 10. Baumgarte position correction, colour by colour ----
      for (int col = 0; col < ncol; ++col) {
        for (int m = L.coloff[col] + lane; m < L.coloff[col + 1]; m += kWave) {
          const uint32_t ab = L.mab[m];
          const int j = (int)(ab & 0xffffu);
          baumgarte_pair(L, (int)(ab >> 16), j, j == (int)kGround, mdev(L, m), a.beta, a.slop);
        }
        wave_sync();
      }
      timer.mark(L, lane, 9);
    }
    // ---- withdrawal of pushed bodies ----
    for (int r = lane; r < np; r += kWave) {
      const int b = L.pb[r];
      if (!(L.pwd[r] > 0.f) || step < (int64_t)L.ps[r] || !(L.flag[b] & kActive) || (L.tfz[L.tw[b]] & 4u)) continue;
      float dx[3], f[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) { dx[k] = L.x[k * NB + b] - L.px0[3 * r + k]; f[k] = L.pf[3 * r + k]; }
      if (dot3(dx, f) >= L.pwd[r] * sqrtf(dot3(f, f))) {
        atomicAnd(&L.flag[b], ~kActive);
#pragma unroll
        for (int k = 0; k < 3; ++k) { L.v[k * NB + b] = 0.f; L.w[k * NB + b] = 0.f; }
      }
    }
    wave_sync();
    // ---- episode criteria at the end of the step (the pack's manifold block is free scratch
    // until the next step's manifolds) ----
    if (kExt && a.ep_state) {
      episode_update(L, a, gt0, gb0, nt, lane, step, L.md);
      wave_sync();
    }
  }

  // ---- write the pack back (a body without mass keeps its stored velocity) ----
  for (int i = lane; i < nb; i += kWave) {
    const int g = gb0 + i;
    const bool dyn = (L.flag[i] & kDynamic) != 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a.x[k * CAP + g] = L.x[k * NB + i];
      if (dyn) {
        a.v[k * CAP + g] = L.v[k * NB + i];
        a.w[k * CAP + g] = L.w[k * NB + i];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) a.q[k * CAP + g] = L.q[k * NB + i];
    const uint32_t f = L.flag[i];
    a.flags[g] = (f & kHeld) ? ((f & ~kHeld) | kActive) : f;
  }
  for (int t = lane; t < nt; t += kWave) {
    const int g = gt0 + t;
#pragma unroll
    for (int k = 0; k < 3; ++k) a.tower_count[4 * g + k] += L.tcnt[4 * t + k];
    a.tower_count[4 * g + 3] = L.tcnt[4 * t + 3];
    a.tower_res[2 * g] = L.tres[2 * t];
    a.tower_res[2 * g + 1] = L.tres[2 * t + 1];
    a.tower_frozen[g] = L.tfz[t] & 1u;
  }
  for (int r = lane; r < np; r += kWave) {
#pragma unroll
    for (int k = 0; k < 3; ++k) a.push_x0[3 * (gp0 + r) + k] = L.px0[3 * r + k];
  }
  if constexpr (kLearned) {
    if (a.warm_start == 2)
      for (int t = lane; t < nt; t += kWave) {
        a.tower_fallback[2 * (gt0 + t)] += L.tfc[2 * t];
        a.tower_fallback[2 * (gt0 + t) + 1] += L.tfc[2 * t + 1];
      }
  }
  if (keep_prev) {
    const int npv = L.scal[4];
    for (int p = lane; p < npv; p += kWave) {
      const int g = slot0 + p;
      a.prev_key[g] = L.pkey[p];
      a.prev_data[16 * g + 3] = __uint_as_float(L.pslot[p]);
#pragma unroll
      for (int k = 0; k < 3; ++k) a.prev_data[16 * g + k] = L.pnrm[k * PC + p];
#pragma unroll
      for (int k = 0; k < 12; ++k) a.prev_data[16 * g + 4 + k] = L.plam[k * PC + p];
    }
    if (lane == 0) a.prev_count[pk] = npv;
  }
  if (lane == 0 && L.scal[3]) {
    a.pack_error[pk] |= (uint32_t)L.scal[3];
    atomicOr(a.err_flag, (uint32_t)L.scal[3]);
  }
  timer.mark(L, lane, 0);
  wave_sync();
  if (a.phase_cycles && lane < kPhases) atomicAdd(&a.phase_cycles[lane], L.cyc[lane]);
}

// ------------------------------------------------------------------------------------------------
// Islands stepped by the whole GPU (Sec. "Discussion and Implications for Anastylosis": site-scale
// walls).  One cooperative launch runs every step; its phases are separated by grid-wide barriers
// and every workgroup passes the same barriers in the same order (all loop bounds below are
// uniform: launch parameters or scalars read after a barrier).  Body indices are 32-bit (the
// ground is -1).  The stages are those of a pack, grid-wide:
//   forces, frames -> uniform-grid broadphase (cells of the largest AABB plus the margin, 27
//   neighbour cells, each body's candidates j > i sorted, the ground last: the canonical list with
//   no per-body cap) -> SAT -> compaction -> partitioned greedy colouring (four passes: inside
//   partitions of `partition` bodies, then between neighbouring partitions even / odd, then the
//   rest, each pass in canonical order; one thread per partition or partition pair) -> colour sort
//   -> manifolds -> PGS colour by colour -> outputs, residual -> integration -> Baumgarte colour
//   by colour -> withdrawal at the end of a step.
// ------------------------------------------------------------------------------------------------
namespace mega {

enum {
  sFrozen = 0, sErr, sNcand, sNman, sNcol, sCand, sMans, sPtsAll,
  sLo = 16, sHi = 19, sHmax = 22,
  sColOff = 32,          // 65 words
  sColCnt = 100,         // 64 words
  sColCur = 168          // 64 words
};

__device__ __forceinline__ uint32_t ford(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float funord(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ Lds view(const MegaArgs& a) {
  Lds L{};
  const int nb = a.nb;
  float* p = a.body;
  L.x = p; L.q = p + 3 * nb; L.v = p + 7 * nb; L.w = p + 10 * nb; L.he = p + 13 * nb;
  L.invm = p + 16 * nb; L.Iw = p + 17 * nb; L.hm = p + 23 * nb;
  L.flag = a.ubody;
  L.tw = reinterpret_cast<int32_t*>(a.ubody + nb);
  L.nbp = nb;
  L.pc = 0;
  return L;
}

// block-wide sums (and a second sum) through LDS; every thread gets the results
__device__ __forceinline__ void block_sum2(int32_t* sh, int32_t* sh2, int& x, int& y) {
  sh[threadIdx.x] = x;
  sh2[threadIdx.x] = y;
  __syncthreads();
  for (int d = kMegaThreads / 2; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
      sh[threadIdx.x] += sh[threadIdx.x + d];
      sh2[threadIdx.x] += sh2[threadIdx.x + d];
    }
    __syncthreads();
  }
  x = sh[0];
  y = sh2[0];
  __syncthreads();
}

// Exclusive prefix sums of v[0, n) in place over the whole grid; returns the total.  Thread t
// scans the run [t per, (t + 1) per); the workgroups' sums go through ired (one barrier inside).
// The caller passes a barrier before anyone reads v.
__device__ int grid_scan(cooperative_groups::grid_group& grid, int32_t* v, int n, int32_t* ired, int32_t* sh,
                         int32_t* sh2) {
  const int T = (int)gridDim.x * kMegaThreads;
  const int gt = (int)blockIdx.x * kMegaThreads + (int)threadIdx.x;
  const int per = (n + T - 1) / T;
  const int lo = min(n, gt * per), hi = min(n, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int d = 1; d < kMegaThreads; d <<= 1) {
    const int t = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  const int incl = sh[threadIdx.x];
  if (threadIdx.x == kMegaThreads - 1) ired[blockIdx.x] = incl;
  __syncthreads();
  grid.sync();
  int before = 0, total = 0;
  for (int b = (int)threadIdx.x; b < (int)gridDim.x; b += kMegaThreads) {
    const int x = ired[b];
    total += x;
    if (b < (int)blockIdx.x) before += x;
  }
  block_sum2(sh, sh2, before, total);
  int run = before + incl - s;
  for (int i = lo; i < hi; ++i) {
    const int c = v[i];
    v[i] = run;
    run += c;
  }
  return total;
}

// the uniform grid of the active bodies' centres: origin, cell size and cells per axis (the same
// on every thread: read from the scalars after a barrier)
struct Grid {
  float lo[3], h;
  int n[3];
  __device__ __forceinline__ int cell_of(const float x[3]) const {
    int c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = min(n[k] - 1, max(0, (int)floorf((x[k] - lo[k]) / h)));
    return (c[2] * n[1] + c[1]) * n[0] + c[0];
  }
};

__device__ __forceinline__ Grid make_grid(const int32_t* S, float margin, int cap) {
  Grid G;
  float hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    G.lo[k] = funord((uint32_t)S[sLo + k]);
    hi[k] = funord((uint32_t)S[sHi + k]);
    if (!(hi[k] >= G.lo[k])) { G.lo[k] = 0.f; hi[k] = 0.f; }   // no active body
  }
  // two bodies whose AABBs (with the margin) overlap are at most this far apart on every axis
  G.h = fmaxf(2.f * funord((uint32_t)S[sHmax]) + margin, 1e-6f);
  bool fits = false;
  for (int it = 0; it < 16 && !fits; ++it) {
    double total = 1.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.n[k] = (int)fminf(floorf((hi[k] - G.lo[k]) / G.h) + 1.f, 1.0e6f);
      total *= (double)G.n[k];
    }
    fits = total <= (double)cap;
    if (!fits) G.h *= (float)fmax(1.01, cbrt(total / (double)cap) * 1.01);
  }
  if (!fits) {
    // one cell (every pair is tested): correct at any size
    G.n[0] = G.n[1] = G.n[2] = 1;
    G.h = 3.0e38f;
  }
  return G;
}

// greedy first fit of canonical pair m = (a, b) over the colour masks of its dynamic bodies
__device__ __forceinline__ void colour_pair(int m, int a, int b, const uint32_t* flag, uint32_t* mlo, uint32_t* mhi,
                                            int32_t* col_of, int32_t* S) {
  const bool da = (flag[a] & kDynamic) != 0, db = b >= 0 && (flag[b] & kDynamic);
  uint64_t u = 0ull;
  if (da) u |= (uint64_t)mlo[a] | ((uint64_t)mhi[a] << 32);
  if (db) u |= (uint64_t)mlo[b] | ((uint64_t)mhi[b] << 32);
  int col = -1;
  if (u != ~0ull) {
    col = __ffsll((unsigned long long)~u) - 1;
    const uint64_t bit = 1ull << col;
    if (da) { mlo[a] |= (uint32_t)bit; mhi[a] |= (uint32_t)(bit >> 32); }
    if (db) { mlo[b] |= (uint32_t)bit; mhi[b] |= (uint32_t)(bit >> 32); }
  } else {
    atomicOr(&S[sErr], (int)kErrCol);
  }
  col_of[m] = col;
}

// one PGS visit of the record at `rec` (pair a, b; b < 0: the ground), one thread
__device__ __forceinline__ void solve_rec(const Lds& L, float* rec, const float* tbp, int a, int b, int np, float mu,
                                          const SolveOpts& o) {
  float r[12], l[12], tb[4];
  const float4* r4 = reinterpret_cast<const float4*>(rec);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float4 x = r4[c], y = r4[3 + c];
    r[4 * c] = x.x; r[4 * c + 1] = x.y; r[4 * c + 2] = x.z; r[4 * c + 3] = x.w;
    l[4 * c] = y.x; l[4 * c + 1] = y.y; l[4 * c + 2] = y.z; l[4 * c + 3] = y.w;
  }
  const float4 nd = r4[6];
  const float4 t4 = o.bias ? *reinterpret_cast<const float4*>(tbp) : make_float4(0.f, 0.f, 0.f, 0.f);
  const float n[3] = {nd.x, nd.y, nd.z};
  tb[0] = o.bias ? t4.x : 0.f; tb[1] = o.bias ? t4.y : 0.f; tb[2] = o.bias ? t4.z : 0.f; tb[3] = o.bias ? t4.w : 0.f;
  const bool ground = b < 0;
  Frame F;
  LBody A, B;
  float dAB[3];
  pair_open(L, a, ground ? 0 : b, ground, n, F, A, B, dAB);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < np) {
      const float rA[3] = {r[3 * j], r[3 * j + 1], r[3 * j + 2]};
      const float rB[3] = {rA[0] + dAB[0], rA[1] + dAB[1], rA[2] + dAB[2]};
      solve_point(A, B, rA, rB, &l[3 * j], mu, o, tb[j]);
    }
  }
  store_local(L, a, F, A);
  if (!ground) store_local(L, b, F, B);
  float4* w4 = reinterpret_cast<float4*>(rec);
#pragma unroll
  for (int c = 0; c < 3; ++c) w4[3 + c] = make_float4(l[4 * c], l[4 * c + 1], l[4 * c + 2], l[4 * c + 3]);
}

}  // namespace mega

__global__ void __launch_bounds__(kMegaThreads) mega_kernel(MegaArgs a) {
  namespace cg = cooperative_groups;
  using namespace mega;
  cg::grid_group grid = cg::this_grid();
  __shared__ int32_t sh[kMegaThreads], sh2[kMegaThreads];
  __shared__ float shf[kMegaThreads], shf2[kMegaThreads];
  // partition walks: colour masks (2 words) and dynamic flags of up to two partitions, pairs
  __shared__ uint32_t lmask[4 * kMegaStagedPartition];
  __shared__ uint8_t ldyn[2 * kMegaStagedPartition];
  __shared__ int32_t lpair[2 * kMegaChunk];
  const int NB = a.nb, CAP = a.cap, CC = a.cand_cap;
  const int gt = (int)blockIdx.x * kMegaThreads + (int)threadIdx.x;
  const int GS = (int)gridDim.x * kMegaThreads;
  const Lds L = view(a);
  int32_t* const S = a.scal;
  uint32_t* const mlo = a.ubody + 2 * NB;
  uint32_t* const mhi = a.ubody + 3 * NB;
  int32_t* const cellof = reinterpret_cast<int32_t*>(a.ubody + 4 * NB);
  int32_t* const ccount = reinterpret_cast<int32_t*>(a.ubody + 5 * NB);   // counts, then offsets
  int32_t* const cellbody = reinterpret_cast<int32_t*>(a.ubody + 7 * NB);
  int32_t* const cstart = a.cells;                     // counts, then first body of each cell
  int32_t* const cfill = a.cells + a.ncell_cap + 1;
  uint32_t* const ca = a.cand;
  uint32_t* const cb = a.cand + CC;
  int32_t* const chit = reinterpret_cast<int32_t*>(a.cand + 2 * CC);
  int32_t* const man_a = a.man;
  int32_t* const man_b = a.man + CC;
  int32_t* const man_col = a.man + 2 * CC;
  int32_t* const man_slot = a.man + 3 * CC;
  int32_t* const s_a = a.man + 4 * CC;
  int32_t* const s_b = a.man + 5 * CC;
  uint32_t* const s_meta = reinterpret_cast<uint32_t*>(a.man + 6 * CC);
  int32_t* const far = a.part + a.nparts + 1;
  const float dt = a.dt;
  const SolveOpts opts = {a.restitution, a.friction_cone != 0, a.restitution_bias != 0};
  const int PS = a.partition;

  // ---- load the island (inverse mass; the inverse inertia is taken where needed) ----
  for (int i = gt; i < NB; i += GS) {
    const int g = a.g0 + i;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      L.x[k * NB + i] = a.x[k * CAP + g];
      L.v[k * NB + i] = a.v[k * CAP + g];
      L.w[k * NB + i] = a.w[k * CAP + g];
      L.he[k * NB + i] = a.he[k * CAP + g];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) L.q[k * NB + i] = a.q[k * CAP + g];
    const float m = a.mass[g];
    const bool dyn = m > 0.f;
    L.invm[i] = dyn ? 1.f / m : 0.f;
    L.flag[i] = a.flags[g];
    L.tw[i] = 0;
    if (!dyn) {
#pragma unroll
      for (int k = 0; k < 3; ++k) { L.v[k * NB + i] = 0.f; L.w[k * NB + i] = 0.f; }
    }
  }
  if (gt == 0) {
    S[sFrozen] = a.tower_frozen[a.tslot] ? 1 : 0;
    S[sErr] = 0;
    S[sCand] = 0; S[sMans] = 0; S[sPtsAll] = 0;
    S[sNcol] = 0;
  }
  grid.sync();
  // a non-finite state freezes the island from the first step on
  for (int i = gt; i < NB; i += GS) {
    if (!(L.flag[i] & kActive)) continue;
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      finite = finite && isfinite(L.x[k * NB + i]) && isfinite(L.v[k * NB + i]) && isfinite(L.w[k * NB + i]);
#pragma unroll
    for (int k = 0; k < 4; ++k) finite = finite && isfinite(L.q[k * NB + i]);
    if (!finite) {
      atomicOr(&S[sFrozen], 1);
      atomicOr(&S[sErr], (int)kErrNan);
    }
  }
  grid.sync();

  for (int s = 0; s < a.n_steps; ++s) {
    const int64_t step = a.step0 + s;
    for (int r = gt; r < a.np; r += GS) {
      const int row = a.p0 + r;
      if ((int64_t)a.push_start[row] == step) {
        const int b = a.push_body[row] - a.g0;
#pragma unroll
        for (int k = 0; k < 3; ++k) a.push_x0[3 * row + k] = L.x[k * NB + b];
      }
    }
    grid.sync();
    for (int sub = 0; sub < a.n_sub; ++sub) {
      if (S[sFrozen]) continue;   // uniform: written before the last barrier only
      const bool last = (s == a.n_steps - 1) && (sub == a.n_sub - 1);
      // ---- 1. external forces and pushes; 2. frames; colour masks cleared ----
      for (int i = gt; i < NB; i += GS) {
        const uint32_t f = L.flag[i];
        const bool moving = (f & (kActive | kDynamic)) == (kActive | kDynamic);
        if (moving) {
          float vv[3];
          load3(L.v, NB, i, vv);
#pragma unroll
          for (int k = 0; k < 3; ++k) vv[k] += dt * a.g[k];
          store3(L.v, NB, i, vv);
        }
        float R[9];
        body_R(L, i, R);
        const float he0 = L.he[i], he1 = L.he[NB + i], he2 = L.he[2 * NB + i];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          L.hm[k * NB + i] = fabsf(R[3 * k]) * he0 + fabsf(R[3 * k + 1]) * he1 + fabsf(R[3 * k + 2]) * he2;
        float d[3];
        if (moving) inv_body_inertia(L, i, a.mass[a.g0 + i], d);
        else d[0] = d[1] = d[2] = 0.f;
        L.Iw[i] = R[0] * d[0] * R[0] + R[1] * d[1] * R[1] + R[2] * d[2] * R[2];
        L.Iw[NB + i] = R[3] * d[0] * R[3] + R[4] * d[1] * R[4] + R[5] * d[2] * R[5];
        L.Iw[2 * NB + i] = R[6] * d[0] * R[6] + R[7] * d[1] * R[7] + R[8] * d[2] * R[8];
        L.Iw[3 * NB + i] = R[0] * d[0] * R[3] + R[1] * d[1] * R[4] + R[2] * d[2] * R[5];
        L.Iw[4 * NB + i] = R[0] * d[0] * R[6] + R[1] * d[1] * R[7] + R[2] * d[2] * R[8];
        L.Iw[5 * NB + i] = R[3] * d[0] * R[6] + R[4] * d[1] * R[7] + R[5] * d[2] * R[8];
        mlo[i] = 0u;
        mhi[i] = 0u;
      }
      // pushes (rows in order; a body's pushes add in row order, as on a pack)
      for (int i = gt; i < NB; i += GS) {
        if ((L.flag[i] & (kActive | kDynamic)) != (kActive | kDynamic)) continue;
        const int g = a.g0 + i;
        for (int r = 0; r < a.np; ++r) {
          const int row = a.p0 + r;
          if (a.push_body[row] == g && step >= (int64_t)a.push_start[row] &&
              step < (int64_t)a.push_start[row] + a.push_steps[row]) {
#pragma unroll
            for (int k = 0; k < 3; ++k) L.v[k * NB + i] += dt * a.push_force[3 * row + k] * L.invm[i];
          }
        }
      }
      if (gt == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) { S[sLo + k] = (int32_t)ford(3.0e38f); S[sHi + k] = (int32_t)ford(-3.0e38f); }
        S[sHmax] = (int32_t)ford(0.f);
        S[sNcol] = 0;
      }
      if (gt < kMaxColours) S[sColCnt + gt] = 0;
      for (int c = gt; c <= a.ncell_cap; c += GS) { cstart[c] = 0; cfill[c] = 0; }
      grid.sync();
      // ---- 3. uniform grid: bounds of the active centres, largest AABB half size ----
      {
        float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f}, hmax = 0.f;
        for (int i = gt; i < NB; i += GS) {
          if (!(L.flag[i] & kActive)) continue;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const float x = L.x[k * NB + i];
            lo[k] = fminf(lo[k], x);
            hi[k] = fmaxf(hi[k], x);
            hmax = fmaxf(hmax, L.hm[k * NB + i]);
          }
        }
        // wave reductions, then one atomic per wave
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], __shfl_xor(lo[k], d));
            hi[k] = fmaxf(hi[k], __shfl_xor(hi[k], d));
          }
          hmax = fmaxf(hmax, __shfl_xor(hmax, d));
        }
        // then across the block's waves in LDS, one atomic per block and quantity
        const int wv = (int)threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
          for (int k = 0; k < 3; ++k) { shf[8 * wv + k] = lo[k]; shf[8 * wv + 3 + k] = hi[k]; }
          shf[8 * wv + 6] = hmax;
        }
        __syncthreads();
        if (threadIdx.x < 7) {
          const int q = (int)threadIdx.x;
          float v = shf[q];
          for (int w2 = 1; w2 < kMegaThreads / kWave; ++w2)
            v = (q < 3) ? fminf(v, shf[8 * w2 + q]) : fmaxf(v, shf[8 * w2 + q]);
          if (q < 3) atomicMin(reinterpret_cast<uint32_t*>(&S[sLo + q]), ford(v));
          else if (q < 6) atomicMax(reinterpret_cast<uint32_t*>(&S[sHi + q - 3]), ford(v));
          else atomicMax(reinterpret_cast<uint32_t*>(&S[sHmax]), ford(v));
        }
        __syncthreads();
      }
      grid.sync();
      const Grid G = make_grid(S, a.margin, a.ncell_cap);
      const int ncell = G.n[0] * G.n[1] * G.n[2];
      for (int i = gt; i < NB; i += GS) {
        int c = -1;
        if (L.flag[i] & kActive) {
          float x[3];
          load3(L.x, NB, i, x);
          c = G.cell_of(x);
          atomicAdd(&cstart[c], 1);
        }
        cellof[i] = c;
      }
      grid.sync();
      const int nin = grid_scan(grid, cstart, ncell, a.ired, sh, sh2);
      if (gt == 0) cstart[ncell] = nin;
      grid.sync();
      for (int i = gt; i < NB; i += GS) {
        const int c = cellof[i];
        if (c >= 0) cellbody[cstart[c] + atomicAdd(&cfill[c], 1)] = i;
      }
      grid.sync();
      // ---- candidates: per body i, the bodies j > i of the 27 neighbour cells that pass
      // Eq. (aabb) with the margin (inclusive), then the ground; counted, placed, written ----
      auto walk = [&](int i, uint32_t* out, int room) -> int {
        int cnt = 0;
        const uint32_t fi = L.flag[i];
        if (!(fi & kActive)) return 0;
        const bool dyni = (fi & kDynamic) != 0;
        float xi[3], hi[3];
        load3(L.x, NB, i, xi);
        load3(L.hm, NB, i, hi);
        int ci[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) ci[k] = min(G.n[k] - 1, max(0, (int)floorf((xi[k] - G.lo[k]) / G.h)));
        for (int dz = -1; dz <= 1; ++dz) {
          const int cz = ci[2] + dz;
          if (cz < 0 || cz >= G.n[2]) continue;
          for (int dy = -1; dy <= 1; ++dy) {
            const int cy = ci[1] + dy;
            if (cy < 0 || cy >= G.n[1]) continue;
            for (int dx = -1; dx <= 1; ++dx) {
              const int cx = ci[0] + dx;
              if (cx < 0 || cx >= G.n[0]) continue;
              const int c = (cz * G.n[1] + cy) * G.n[0] + cx;
              for (int k = cstart[c]; k < cstart[c + 1]; ++k) {
                const int j = cellbody[k];
                if (j <= i) continue;
                const uint32_t fj = L.flag[j];
                if (!(fj & kActive) || !(dyni || (fj & kDynamic))) continue;
                if (fabsf(xi[0] - L.x[j]) <= hi[0] + L.hm[j] + a.margin &&
                    fabsf(xi[1] - L.x[NB + j]) <= hi[1] + L.hm[NB + j] + a.margin &&
                    fabsf(xi[2] - L.x[2 * NB + j]) <= hi[2] + L.hm[2 * NB + j] + a.margin) {
                  if (out && cnt < room) out[cnt] = (uint32_t)j;
                  ++cnt;
                }
              }
            }
          }
        }
        if (out) {
          // ascending j (insertion sort of the body's own run)
          const int n = min(cnt, room);
          for (int p = 1; p < n; ++p) {
            const uint32_t v = out[p];
            int q = p - 1;
            while (q >= 0 && out[q] > v) { out[q + 1] = out[q]; --q; }
            out[q + 1] = v;
          }
        }
        if (dyni && (xi[2] - hi[2] <= a.margin)) {
          if (out && cnt < room) out[cnt] = ~0u;
          ++cnt;
        }
        return cnt;
      };
      for (int i = gt; i < NB; i += GS) ccount[i] = walk(i, nullptr, 0);
      grid.sync();
      const int ncand_all = grid_scan(grid, ccount, NB, a.ired, sh, sh2);
      if (gt == 0) S[sNcand] = min(ncand_all, CC);
      grid.sync();
      // a body whose run does not fit the candidate capacity ends the list before its run
      for (int i = gt; i < NB; i += GS) {
        const int off = ccount[i], end = i + 1 < NB ? ccount[i + 1] : ncand_all;
        if (end > CC && off <= CC) {
          atomicMin(&S[sNcand], off);
          atomicOr(&S[sErr], (int)kErrCand);
        }
      }
      grid.sync();
      const int ncand = S[sNcand];
      for (int i = gt; i < NB; i += GS) {
        const int off = ccount[i], end = i + 1 < NB ? ccount[i + 1] : ncand_all;
        if (end > ncand || end == off) continue;
        walk(i, cb + off, end - off);
        for (int k = off; k < end; ++k) ca[k] = (uint32_t)i;
      }
      grid.sync();
      // ---- 4. narrowphase (SAT, Sec. "Narrowphase: OBB SAT"; the ground: a vertex below z = 0) ----
      for (int k = gt; k < ncand; k += GS) {
        const int i = (int)ca[k];
        const uint32_t jb = cb[k];
        bool hit;
        if (jb == ~0u) {
          hit = L.x[2 * NB + i] - L.hm[2 * NB + i] < 0.f;
        } else {
          const int j = (int)jb;
          float RA[9], RB[9], heA[3], heB[3], d[3], n[3], depth;
          body_R(L, i, RA);
          body_R(L, j, RB);
          load3(L.he, NB, i, heA);
          load3(L.he, NB, j, heB);
#pragma unroll
          for (int q = 0; q < 3; ++q) d[q] = L.x[q * NB + j] - L.x[q * NB + i];
          hit = sat_boxes(RA, heA, RB, heB, d, n, depth);
        }
        chit[k] = hit ? 1 : 0;
      }
      grid.sync();
      const int nman = grid_scan(grid, chit, ncand, a.ired, sh, sh2);
      if (gt == 0) S[sNman] = nman;
      grid.sync();
      for (int k = gt; k < ncand; k += GS) {
        const int pos = chit[k], nxt = k + 1 < ncand ? chit[k + 1] : nman;
        if (nxt > pos) {
          man_a[pos] = (int32_t)ca[k];
          man_b[pos] = cb[k] == ~0u ? -1 : (int32_t)cb[k];
          man_col[pos] = -1;
        }
      }
      grid.sync();
      // ---- 5. partitioned greedy colouring ----
      for (int p = gt; p <= a.nparts; p += GS) {
        // the first canonical pair whose first body is in partition p or later
        const int key = (int)min((int64_t)p * PS, (int64_t)NB);
        int lo = 0, hi = nman;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (man_a[mid] < key) lo = mid + 1; else hi = mid;
        }
        a.part[p] = lo;
        if (p < a.nparts) far[p] = 0;
      }
      grid.sync();
      if (PS <= kMegaStagedPartition) {
        // one workgroup per partition (pass 1) or partition pair (passes 2, 3): the bodies' colour
        // masks and dynamic flags and the pairs, in chunks, staged in LDS; its first thread walks them
        for (int pass = 0; pass < 3; ++pass) {
          for (int p = (int)blockIdx.x; p < a.nparts; p += (int)gridDim.x) {
            if (pass > 0 && (p & 1) != pass - 1) continue;
            const int b0 = p * PS, nbp = min((pass == 0 ? 1 : 2) * PS, NB - b0);
            for (int i = (int)threadIdx.x; i < nbp; i += kMegaThreads) {
              lmask[2 * i] = mlo[b0 + i];
              lmask[2 * i + 1] = mhi[b0 + i];
              ldyn[i] = (L.flag[b0 + i] & kDynamic) ? 1 : 0;
            }
            int nfar = 0;
            for (int c0 = a.part[p]; c0 < a.part[p + 1]; c0 += kMegaChunk) {
              const int n = min(kMegaChunk, a.part[p + 1] - c0);
              __syncthreads();
              for (int k = (int)threadIdx.x; k < n; k += kMegaThreads) {
                lpair[2 * k] = man_a[c0 + k] - b0;
                lpair[2 * k + 1] = man_b[c0 + k];
              }
              __syncthreads();
              if (threadIdx.x == 0) {
                for (int k = 0; k < n; ++k) {
                  // the second body's place: the ground or this partition (0), the next (1), further (2)
                  const int i = lpair[2 * k], jg = lpair[2 * k + 1];
                  const int j = jg < 0 ? -1 : jg - b0;
                  const int where = j < PS ? 0 : (j < 2 * PS ? 1 : 2);
                  if (pass == 0 && where == 2) ++nfar;
                  if (where != (pass == 0 ? 0 : 1)) continue;
                  const bool da = ldyn[i] != 0, db = j >= 0 && ldyn[j] != 0;
                  uint64_t u = 0ull;
                  if (da) u |= (uint64_t)lmask[2 * i] | ((uint64_t)lmask[2 * i + 1] << 32);
                  if (db) u |= (uint64_t)lmask[2 * j] | ((uint64_t)lmask[2 * j + 1] << 32);
                  int col = -1;
                  if (u != ~0ull) {
                    col = __ffsll((unsigned long long)~u) - 1;
                    const uint64_t bit = 1ull << col;
                    if (da) { lmask[2 * i] |= (uint32_t)bit; lmask[2 * i + 1] |= (uint32_t)(bit >> 32); }
                    if (db) { lmask[2 * j] |= (uint32_t)bit; lmask[2 * j + 1] |= (uint32_t)(bit >> 32); }
                  } else {
                    atomicOr(&S[sErr], (int)kErrCol);
                  }
                  man_col[c0 + k] = col;
                }
              }
            }
            __syncthreads();
            for (int i = (int)threadIdx.x; i < nbp; i += kMegaThreads) {
              mlo[b0 + i] = lmask[2 * i];
              mhi[b0 + i] = lmask[2 * i + 1];
            }
            if (pass == 0 && threadIdx.x == 0) far[p] = nfar;
            __syncthreads();
          }
          grid.sync();
        }
      } else {
        // partitions too large to stage: one thread per partition (pair), from device memory
        for (int pass = 0; pass < 3; ++pass) {
          for (int p = gt; p < a.nparts; p += GS) {
            if (pass > 0 && (p & 1) != pass - 1) continue;
            for (int m = a.part[p]; m < a.part[p + 1]; ++m) {
              const int i = man_a[m], j = man_b[m];
              const int pj = j < 0 ? p : j / PS;
              if (pass == 0 && pj > p + 1) ++far[p];
              if ((pass == 0 && pj == p) || (pass > 0 && pj == p + 1)) colour_pair(m, i, j, L.flag, mlo, mhi, man_col, S);
            }
          }
          grid.sync();
        }
      }
      // the pairs between partitions further apart: one thread, canonical order
      if (gt == 0) {
        for (int p = 0; p < a.nparts; ++p) {
          if (far[p] == 0) continue;
          for (int m = a.part[p]; m < a.part[p + 1]; ++m) {
            const int i = man_a[m], j = man_b[m];
            if (j >= 0 && j / PS > p + 1) colour_pair(m, i, j, L.flag, mlo, mhi, man_col, S);
          }
        }
      }
      grid.sync();
      // colour-sorted slots (the order inside a colour is free: its pairs share no dynamic body):
      // each workgroup counts the colours of a contiguous run of the canonical list in LDS (ranks
      // from LDS atomics), adds its counts once per colour, and takes a range of every colour
      const int chunk = (nman + (int)gridDim.x - 1) / (int)gridDim.x;
      const int cm0 = min(nman, (int)blockIdx.x * chunk), cm1 = min(nman, cm0 + chunk);
      if (threadIdx.x < kMaxColours) sh[threadIdx.x] = 0;
      __syncthreads();
      for (int m = cm0 + (int)threadIdx.x; m < cm1; m += kMegaThreads) {
        const int c = man_col[m];
        man_slot[m] = c >= 0 ? atomicAdd(&sh[c], 1) : -1;
      }
      __syncthreads();
      if (threadIdx.x < kMaxColours && sh[threadIdx.x] > 0) atomicAdd(&S[sColCnt + threadIdx.x], sh[threadIdx.x]);
      grid.sync();
      if (gt == 0) {
        int off = 0, ncol = 0;
        for (int c = 0; c < kMaxColours; ++c) {
          const int n = S[sColCnt + c];
          S[sColOff + c] = off;
          S[sColCur + c] = 0;
          off += n;
          if (n > 0) ncol = c + 1;
        }
        S[sColOff + kMaxColours] = off;
        S[sNcol] = ncol;
      }
      grid.sync();
      const int ncol = S[sNcol];
      if (threadIdx.x < kMaxColours)
        sh2[threadIdx.x] = sh[threadIdx.x] > 0 ? S[sColOff + threadIdx.x] + atomicAdd(&S[sColCur + threadIdx.x], sh[threadIdx.x])
                                               : 0;
      __syncthreads();
      for (int m = cm0 + (int)threadIdx.x; m < cm1; m += kMegaThreads) {
        const int c = man_col[m];
        int slot = -1;
        if (c >= 0) {
          slot = sh2[c] + man_slot[m];
          s_a[slot] = man_a[m];
          s_b[slot] = man_b[m];
        }
        man_slot[m] = slot;
      }
      grid.sync();
      // ---- 6. manifolds into the colour-sorted slots (zero initial impulses) ----
      {
        int pts = 0, kept = 0;
        for (int m = gt; m < nman; m += GS) {
          const int slot = man_slot[m];
          if (slot < 0) continue;
          const int i = man_a[m], j = man_b[m];
          const bool ground = j < 0;
          float* rec = a.md + (size_t)slot * kManDevWords;
          float n[3], depth;
          uint32_t slots;
          const int np = manifold_geometry<true>(L, i, ground ? 0 : j, ground, a.manifold_mode, rec, n, depth, slots,
                                                 nullptr);
#pragma unroll
          for (int k = 0; k < 12; ++k) rec[12 + k] = 0.f;
          if (a.restitution_bias)
            bias_targets(L, i, ground ? 0 : j, ground, rec, a.mtb + 4 * (size_t)slot, np, n, a.g, dt, a.restitution);
#pragma unroll
          for (int k = 0; k < 3; ++k) rec[24 + k] = n[k];
          rec[27] = depth;
          s_meta[slot] = (uint32_t)np | (slots << 12);
          pts += np;
          kept += 1;
        }
        block_sum2(sh, sh2, pts, kept);
        if (threadIdx.x == 0 && (pts || kept)) {
          atomicAdd(&S[sPtsAll], pts);
          atomicAdd(&S[sMans], kept);
        }
        if (gt == 0) atomicAdd(&S[sCand], ncand);
      }
      grid.sync();
      // ---- 7. PGS sweeps, colour by colour (Sec. "Contact Solver --- Projected Gauss-Seidel") ----
      for (int it = 0; it < a.iters; ++it) {
        for (int c = 0; c < ncol; ++c) {
          const int c1 = S[sColOff + c + 1];
          for (int slot = S[sColOff + c] + gt; slot < c1; slot += GS)
            solve_rec(L, a.md + (size_t)slot * kManDevWords, a.mtb + 4 * (size_t)slot, s_a[slot], s_b[slot],
                      (int)(s_meta[slot] & 15u), a.mu, opts);
          grid.sync();
        }
      }
      // ---- contacts of the launch's last step (canonical order) ----
      if (last) {
        for (int m = gt; m < nman; m += GS) {
          const int slot = man_slot[m];
          a.out_a[m] = man_a[m];
          a.out_b[m] = man_b[m];
          if (slot < 0) {
            a.out_meta[m] = 0u;
            continue;
          }
          const float* rec = a.md + (size_t)slot * kManDevWords;
          const uint32_t meta = s_meta[slot];
          const int np = (int)(meta & 15u);
          a.out_meta[m] = (meta & 0x0ffff00fu) | ((uint32_t)man_col[m] << 4);
          const float nn[3] = {rec[24], rec[25], rec[26]};
          Frame F;
          make_frame(nn, F);
          for (int k = 0; k < 3; ++k) {
            a.out_geo[8 * (size_t)m + k] = nn[k];
            a.out_geo[8 * (size_t)m + 3 + k] = F.f[1][k];
          }
          a.out_geo[8 * (size_t)m + 6] = rec[27];
          a.out_geo[8 * (size_t)m + 7] = 0.f;
          const int ia = man_a[m];
          for (int q = 0; q < 4; ++q) {
            float rl[3] = {0.f, 0.f, 0.f}, rw[3];
            if (q < np)
              for (int k = 0; k < 3; ++k) rl[k] = rec[q * 3 + k];
            to_world(F, rl, rw);
            for (int k = 0; k < 3; ++k) {
              a.out_pts[24 * (size_t)m + 6 * q + k] = L.x[k * NB + ia] + rw[k];
              a.out_pts[24 * (size_t)m + 6 * q + 3 + k] = q < np ? rec[12 + q * 3 + k] : 0.f;
            }
          }
        }
        if (gt == 0) *a.out_count = nman;
      }
      // ---- 8. residual (R21): canonical order, a fixed summation order for a grid size ----
      {
        float sum = 0.f, mx = 0.f;
        int pts = 0, unused = 0;
        for (int m = gt; m < nman; m += GS) {
          const int slot = man_slot[m];
          if (slot < 0) continue;
          float s2, m2;
          const int j = man_b[m];
          const int np = (int)(s_meta[slot] & 15u);
          residual_rec(L, a.md + (size_t)slot * kManDevWords, a.mtb + 4 * (size_t)slot, man_a[m], j < 0 ? 0 : j, j < 0,
                       np, a.mu, opts, s2, m2);
          sum += s2;
          mx = fmaxf(mx, m2);
          pts += np;
        }
        shf[threadIdx.x] = sum;
        shf2[threadIdx.x] = mx;
        __syncthreads();
        for (int d = kMegaThreads / 2; d > 0; d >>= 1) {
          if ((int)threadIdx.x < d) {
            shf[threadIdx.x] += shf[threadIdx.x + d];
            shf2[threadIdx.x] = fmaxf(shf2[threadIdx.x], shf2[threadIdx.x + d]);
          }
          __syncthreads();
        }
        block_sum2(sh, sh2, pts, unused);
        if (threadIdx.x == 0) {
          a.red[2 * blockIdx.x] = shf[0];
          a.red[2 * blockIdx.x + 1] = shf2[0];
          a.ired[blockIdx.x] = pts;
        }
      }
      grid.sync();
      if (gt == 0) {
        float sum = 0.f, mx = 0.f;
        int pts = 0;
        for (int b = 0; b < (int)gridDim.x; ++b) {
          sum += a.red[2 * b];
          mx = fmaxf(mx, a.red[2 * b + 1]);
          pts += a.ired[b];
        }
        const int rows = 3 * pts;
        a.tower_res[2 * a.tslot] = rows ? sqrtf(sum / (float)rows) : 0.f;
        a.tower_res[2 * a.tslot + 1] = mx;
        a.tower_count[4 * a.tslot + 3] = (uint32_t)ncol;
      }
      // ---- 9. integration ----
      for (int i = gt; i < NB; i += GS) {
        if ((L.flag[i] & (kActive | kDynamic)) != (kActive | kDynamic)) continue;
        if (!integrate_body(L, i, a.mass[a.g0 + i], dt)) {
          atomicOr(&S[sErr], (int)kErrNan);
          atomicOr(&S[sFrozen], 1);   // frozen from the next substep on
        }
      }
      grid.sync();
      // ---- 10. Baumgarte position correction (Eq. (baumgarte)), colour by colour ----
      for (int c = 0; c < ncol; ++c) {
        const int c1 = S[sColOff + c + 1];
        for (int slot = S[sColOff + c] + gt; slot < c1; slot += GS) {
          const int j = s_b[slot];
          baumgarte_pair(L, s_a[slot], j < 0 ? 0 : j, j < 0, a.md + (size_t)slot * kManDevWords, a.beta, a.slop);
        }
        grid.sync();
      }
    }
    // ---- withdrawal of pushed bodies at the end of the step ----
    if (!S[sFrozen]) {
      for (int r = gt; r < a.np; r += GS) {
        const int row = a.p0 + r;
        const int b = a.push_body[row] - a.g0;
        if (!(a.push_withdraw[row] > 0.f) || step < (int64_t)a.push_start[row] || !(L.flag[b] & kActive)) continue;
        float dx[3], f[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) { dx[k] = L.x[k * NB + b] - a.push_x0[3 * row + k]; f[k] = a.push_force[3 * row + k]; }
        if (dot3(dx, f) >= a.push_withdraw[row] * sqrtf(dot3(f, f))) {
          atomicAnd(&L.flag[b], ~kActive);
#pragma unroll
          for (int k = 0; k < 3; ++k) { L.v[k * NB + b] = 0.f; L.w[k * NB + b] = 0.f; }
        }
      }
    }
    grid.sync();
  }

  // ---- write the island back (a body without mass keeps its stored velocity) ----
  for (int i = gt; i < NB; i += GS) {
    const int g = a.g0 + i;
    const bool dyn = (L.flag[i] & kDynamic) != 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a.x[k * CAP + g] = L.x[k * NB + i];
      if (dyn) {
        a.v[k * CAP + g] = L.v[k * NB + i];
        a.w[k * CAP + g] = L.w[k * NB + i];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) a.q[k * CAP + g] = L.q[k * NB + i];
    a.flags[g] = L.flag[i];
  }
  if (gt == 0) {
    a.tower_count[4 * a.tslot + 0] += (uint32_t)S[sCand];
    a.tower_count[4 * a.tslot + 1] += (uint32_t)S[sMans];
    a.tower_count[4 * a.tslot + 2] += (uint32_t)S[sPtsAll];
    a.tower_frozen[a.tslot] = S[sFrozen] ? 1u : 0u;
    if (S[sErr]) {
      atomicOr(a.err_flag, (uint32_t)S[sErr]);
      atomicOr(a.island_err, (uint32_t)S[sErr]);
    }
  }
}

}  // namespace

namespace {

// The dynamic-LDS limit of every variant, once per device (the current one), under a lock so
// that worlds stepped from several host threads agree.
int ensure_lds_limit() {
  static std::mutex attr_mutex;
  static bool attr_set[kMaxDevices] = {};
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev)) return (int)e;
  if (dev < 0 || dev >= kMaxDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(attr_mutex);
  if (!attr_set[dev]) {
    const void* variants[11] = {
        (const void*)step_kernel<false, false, false, false>, (const void*)step_kernel<false, false, false, true>,
        (const void*)step_kernel<true, false, false, true>,   (const void*)step_kernel<false, true, false, false>,
        (const void*)step_kernel<false, true, false, true>,   (const void*)step_kernel<true, true, false, true>,
        (const void*)step_kernel<false, true, true, false>,   (const void*)step_kernel<false, true, true, true>,
        (const void*)step_kernel<true, true, true, true>,
        (const void*)step_kernel<false, false, false, false, true>,
        (const void*)step_kernel<false, false, false, true, true>};
    for (const void* f : variants)
      if (hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024))
        return (int)e;
    attr_set[dev] = true;
  }
  return 0;
}

}  // namespace

int step_launch_config(const StepArgs& a, const void** func, unsigned* block_threads) {
  if (int e = ensure_lds_limit()) return e;
  const bool learned = a.warm_start == 2 || a.feat_out;
  // the variants and the episode criteria run in their own instantiations (the network's kernel
  // always carries them)
  const bool ext = a.friction_cone || a.restitution_bias || a.manifold_mode || a.ep_state;
  const void* f;
  unsigned threads = kWave;
  if (a.in_gmem) {
    if (a.hot_bodies)
      f = learned ? (const void*)step_kernel<true, true, true, true>
                  : (ext ? (const void*)step_kernel<false, true, true, true> : (const void*)step_kernel<false, true, true, false>);
    else
      f = learned ? (const void*)step_kernel<true, true, false, true>
                  : (ext ? (const void*)step_kernel<false, true, false, true> : (const void*)step_kernel<false, true, false, false>);
    threads = learned ? step_threads<true, true>() : step_threads<false, true>();
  } else if (a.lat && !learned) {
    f = ext ? (const void*)step_kernel<false, false, false, true, true> : (const void*)step_kernel<false, false, false, false, true>;
    threads = step_threads<false, false, true>();
  } else {
    f = learned ? (const void*)step_kernel<true, false, false, true>
                : (ext ? (const void*)step_kernel<false, false, false, true> : (const void*)step_kernel<false, false, false, false>);
  }
  *func = f;
  *block_threads = threads;
  return 0;
}

int launch_step(const StepArgs& a, size_t lds_bytes, void* stream) {
  const void* f = nullptr;
  unsigned threads = 0;
  if (int e = step_launch_config(a, &f, &threads)) return e;
  void* args[1] = {const_cast<StepArgs*>(&a)};
  return (int)hipLaunchKernel(f, dim3(a.n_packs), dim3(threads), args, lds_bytes, (hipStream_t)stream);
}

}  // namespace jg

namespace jg {

int mega_blocks(int bodies, int* blocks) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, mega_kernel, kMegaThreads, 0);
  if (e != hipSuccess) return (int)e;
  const int most = std::max(1, std::min(per, 2)) * std::max(1, cus);
  // a grid-wide barrier costs about 0.1 us per workgroup (their arrivals are serialised), a colour
  // of the sweeps about 1.4 us per round of visits: about one workgroup per 3,072 bodies keeps
  // a colour (about a quarter of the bodies in pairs) to a few rounds
  *blocks = std::min(most, std::max(4, (bodies + 3071) / 3072));
  return 0;
}

int launch_mega(const MegaArgs& a, int blocks, void* stream) {
  MegaArgs args = a;
  void* params[] = {(void*)&args};
  return (int)hipLaunchCooperativeKernel((const void*)mega_kernel, dim3((unsigned)blocks), dim3(kMegaThreads), params, 0,
                                         (hipStream_t)stream);
}

}  // namespace jg
