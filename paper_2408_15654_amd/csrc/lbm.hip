// HIP kernels and C ABI of the coupled three-field lattice Boltzmann library
// (phase field f, surfactant g, flow h; arXiv:2408.15654), for gfx950.
//
// State on the device (one caller-owned workspace per simulation).  Two
// copies (ping-pong) of:
//   populations  row-interleaved: lattice row y holds the FG block (for
//                i = 0..8, nx pairs (f_i, g_i), so the two populations that
//                stream from the same source site arrive in one access) and
//                then the H block (h_1..h_8, nx each; h_0 is never read:
//                column 0 of M is e_0 and rows 1-8 of M^-1 start with 0).
//                f_i and g_i are stored as deviations f_i - w_i phi and
//                g_i - w_i psi from the rest values of the writing site;
//   rest         one record per site, (phi, psi) of the same time level:
//                the bases of those deviations;
// plus, updated in place (each site reads and writes only its own entry):
//   aux          one record per site, (ux, uy) of the previous time level
//                (the first-order time differences need it; the previous
//                level's mass flux S is recomputed from the previous phi
//                of the rest records); with a prescribed velocity, u itself;
//   scratch      float64 planes (plane-major) for host transfers and
//                read-back.
// Storage: float64, float32, or float16 deviations with per-field
// power-of-two scales; with float16 storage h is also stored as deviations,
// from 3 w_k (P + c_k . rho u) of the writing site, the rest record carries
// (phi, psi, P, rho ux, rho uy) in float32, and the previous velocity is
// rho u / rho(phi) of that record (aux holds only a prescribed velocity).
//
// One time step is ONE launch of lbm_step_kernel.  Each wavefront owns a
// strip of columns, 60 with one column per lane or 124 with two (float32
// and float16 storage, even nx), plus two halo columns on each side, and
// walks down a tile of rows.  For each row it pulls the f and g deviations
// of the NEXT row, rebuilds that row's phi, psi (and sigma(psi)) from them
// and the rest values of their source sites, keeps a three-row window of
// phi, psi, sigma in registers and takes x-neighbours from adjacent lanes
// with cross-lane moves, so the 9-point stencils need no LDS and no
// barrier.  The h populations and the previous level are read for the
// current row only, and every population is written once.  Workgroups walk
// the tiles in one contiguous band per XCD.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "lbm.h"
#include "lbm_device.h"
#include "arena.h"

using namespace lbm;

namespace {

constexpr int kWave = 64;
constexpr int kPlanes = 26;
constexpr int kScratch = 8;
constexpr int kReduceBlocks = 1024;
constexpr int kReduceVals = 8;

// Minimum waves per SIMD the compiler schedules the step kernel for.  The
// value steers the instruction scheduler as much as the register budget:
// measured on the 2048x2048 many-drop field, 1 (no constraint) is best for
// float64 and float32 storage, 2 for float16 storage (3 spills), and 4
// spills for all.
#ifndef LBM_WAVES_F64
#define LBM_WAVES_F64 1
#endif
#ifndef LBM_WAVES_F32
#define LBM_WAVES_F32 1
#endif
#ifndef LBM_WAVES_F16
#define LBM_WAVES_F16 2
#endif

// Cache policies of the step kernel's stores (the precision structs pick
// one): non-temporal (what a step writes is read again only by the next
// step, long after it has left the caches) or the default.  Measured on the
// 2048x2048 field: non-temporal is 3% faster for float32 storage and 6% for
// float64, the default 4% faster for float16 storage.  A single simulation
// whose step traffic fits the 256 MB Infinity Cache takes default stores in
// every precision (F64C, F32C; cache_resident).
constexpr int kStoreNT = 2;
constexpr int kStoreDefault = 0;

// Storage precisions: S population type, A type of phi/psi/u/S planes,
// R arithmetic type, SCALED: populations carry power-of-two scales.
struct F64 {
  using S = double;
  using A = double;
  using R = double;
  static constexpr bool SCALED = false;
  static constexpr int kMinWaves = LBM_WAVES_F64;  // step kernel waves per SIMD
  static constexpr int kBlockWaves = 4;  // step kernel wavefronts per workgroup
  static constexpr int kStorePol = kStoreNT;  // step kernel store cache policy
  static constexpr bool HDEV = false;  // h stored raw
  static constexpr int kRest = 2;      // rest record: phi, psi
  static constexpr int kAux = 2;       // aux record: ux, uy
};
struct F32 {
  using S = float;
  using A = float;
  using R = float;
  static constexpr bool SCALED = false;
  static constexpr int kMinWaves = LBM_WAVES_F32;  // step kernel waves per SIMD
  static constexpr int kBlockWaves = 4;  // step kernel wavefronts per workgroup
  static constexpr int kStorePol = kStoreNT;  // step kernel store cache policy
  static constexpr bool HDEV = false;
  static constexpr int kRest = 2;
  static constexpr int kAux = 2;
};
struct F16 {
  using S = _Float16;
  using A = float;
  using R = float;
  static constexpr bool SCALED = true;
  static constexpr int kMinWaves = LBM_WAVES_F16;  // step kernel waves per SIMD
  // one wavefront per workgroup: 3% faster than four on the 2048x2048 field
  // (float32 and float64 storage: equal, or slower with one)
  static constexpr int kBlockWaves = 1;
  static constexpr int kStorePol = kStoreDefault;  // step kernel store cache policy
  // h_k stored as deviations from 3 w_k (P + c_k . rho u) of the storing
  // site; P and rho u join phi, psi in the rest record, and the previous
  // velocity is rho u / rho(phi) of that record, so the Navier-Stokes step
  // reads no aux record (it holds only a prescribed velocity).
  static constexpr bool HDEV = true;
  static constexpr int kRest = 5;  // rest record: phi, psi, P, rho ux, rho uy
  static constexpr int kAux = 2;   // aux record: ux, uy (prescribed flow only)
};
// The same storage with default stores: what one step writes is then read
// by the next one from the Infinity Cache while the simulation fits it.
struct F64C : F64 {
  static constexpr int kStorePol = kStoreDefault;
};
struct F32C : F32 {
  static constexpr int kStorePol = kStoreDefault;
};

template <class P>
struct Scales {
  typename P::R f, g, h;     // multiply before storing
  typename P::R fi, gi, hi;  // multiply after loading
};

// Buffer-resource memory access for the step kernel: the address is a
// wave-uniform resource (SGPRs) plus a uniform byte offset (SGPR) plus one
// per-lane 32-bit byte offset (VGPR), so no per-lane 64-bit address math.
// The third dword 0x00020000 is the raw 32-bit-element format of gfx9-family
// buffer descriptors.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
using rsrc_t = __amdgpu_buffer_rsrc_t;

// Guards around a buffer store of more than 64 bits.  Such a store reads
// its data registers over several cycles after it issues; measured on
// gfx950, registers rewritten by the very next instructions (the compiler
// leaves no gap when the store's offset is an SGPR) reached memory with
// the new values in the last lanes of each 16-lane group.  The store is
// pinned between two scheduling barriers and followed by two wait states.
__device__ __forceinline__ void wide_store_begin() { __builtin_amdgcn_sched_barrier(0); }
__device__ __forceinline__ void wide_store_guard() {
  __asm__ volatile("s_nop 1" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
}

// Byte offset of a lane whose buffer stores must not land.  The hardware
// discards a buffer store whose offset is past the resource's range: it
// checks soffset + voffset (+ 4 per further dword) against the resource's
// byte count, without 32-bit wraparound (measured on MI355X for offsets up
// to 0xFFFFFFF0 with soffset 0 to 2^31), and no memory request is made.
// Every resource of the step covers at most kDropped bytes (lbm_create
// checks it), so kDropped, and kDropped plus the few bytes added within a
// record (at most 32, below 2^32 still), is past all of them.
constexpr unsigned kDropped = 0xFFFFFF00u;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, int(bytes),
                                           0x00020000);
}

template <class T>
struct BufIO;
template <>
struct BufIO<float> {
  static __device__ __forceinline__ float load(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  template <int POL>
  static __device__ __forceinline__ void store(float x, rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, POL);
  }
};
template <>
struct BufIO<double> {
  static __device__ __forceinline__ double load(rsrc_t r, unsigned v, unsigned s) {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0);
    const unsigned w0 = w[0], w1 = w[1];
    return __hiloint2double(int(w1), int(w0));
  }
  template <int POL>
  static __device__ __forceinline__ void store(double x, rsrc_t r, unsigned v, unsigned s) {
    u32x2 w;
    w[0] = unsigned(__double2loint(x));
    w[1] = unsigned(__double2hiint(x));
    __builtin_amdgcn_raw_buffer_store_b64(w, r, v, s, POL);
  }
};
template <>
struct BufIO<_Float16> {
  static __device__ __forceinline__ _Float16 load(rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
  }
};

// Population load through a buffer resource, with the float16 scale where
// the storage is scaled; store of an unscaled (float32/float64) one.
template <class P>
__device__ __forceinline__ typename P::R bld(rsrc_t r, unsigned v, unsigned s,
                                             typename P::R inv) {
#pragma clang fp contract(off)
  using R = typename P::R;
  if constexpr (P::SCALED)
    return R(BufIO<typename P::S>::load(r, v, s)) * inv;
  else
    return R(BufIO<typename P::S>::load(r, v, s));
}
template <class P>
__device__ __forceinline__ void bst(typename P::R x, rsrc_t r, unsigned v, unsigned s) {
  static_assert(!P::SCALED, "float16 populations are stored packed (halves_sr)");
  BufIO<typename P::S>::template store<P::kStorePol>(typename P::S(x), r, v, s);
}

template <class P>
__device__ __forceinline__ typename P::R ld(const typename P::S *p, long long i,
                                            typename P::R inv) {
  using R = typename P::R;
  if constexpr (P::SCALED)
    return R(p[i]) * inv;
  else
    return R(p[i]);
}
template <class P>
__device__ __forceinline__ void st(typename P::S *p, long long i, typename P::R v,
                                   typename P::R scale) {
  using S = typename P::S;
  if constexpr (P::SCALED)
    p[i] = S(v * scale);
  else
    p[i] = S(v);
}

template <class P>
struct StepArgs {
  Phys<typename P::R> p;
  Scales<P> sc;
  const typename P::S *src;
  const typename P::A *src_rest;
  typename P::S *dst;
  typename P::A *dst_rest;
  typename P::A *aux;
  int *flag;
  int nx, ny, walls;
  int nstrips, rows;
  int tail_rows, tail_h;  // single-grid launches: short chunks at each band's end
};

// Row offsets and wall flags for pulling row y.
struct RowIdx {
  long long rc, rm, rp;  // offsets of rows y, y-1, y+1 (valid even at walls)
  bool bot, top;         // row y touches the bottom / top wall
};

__device__ __forceinline__ RowIdx row_index(int y, int nx, int ny, int walls) {
  RowIdx r;
  int ym = y - 1, yp = y + 1;
  r.bot = walls && y == 0;
  r.top = walls && y == ny - 1;
  if (ym < 0) ym = walls ? y : ym + ny;
  if (yp >= ny) yp = walls ? y : yp - ny;
  r.rc = (long long)y * nx;
  r.rm = (long long)ym * nx;
  r.rp = (long long)yp * nx;
  return r;
}

// Row y of the lattice for a row index that may lie one or two rows
// outside: periodic wrap, or clamped between walls (clamped rows are only
// read where the bounce-back makes their value irrelevant).
__device__ __forceinline__ int wrap_row(int y, int ny, int walls) {
  if (walls) return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
  return y < 0 ? y + ny : (y >= ny ? y - ny : y);
}

// ------------------------------------------------------------------
// Memory layout (row-interleaved; x fastest inside each block).  Row y of
// the population group holds, in units of the storage type S:
//   block FG: for i = 0..8, nx pairs (f_i, g_i)      -> 18 nx values
//   block H:  for i = 1..8, nx values h_i             ->  8 nx values
// so f_i and g_i, which stream from the same source site, arrive in one
// load.  The rest group holds (phi, psi) pairs and the aux group (ux, uy)
// pairs, one per site.
__device__ __forceinline__ long long fg_idx(int i, int c, int y, int x, int nx) {
  return (long long)y * (kPlanes * nx) + (long long)(i * nx + x) * 2 + c;
}
__device__ __forceinline__ long long h_idx(int i, int y, int x, int nx) {
  return (long long)y * (kPlanes * nx) + 18LL * nx + (long long)(i - 1) * nx + x;
}
template <class P>
__device__ __forceinline__ long long rest_idx(int c, int y, int x, int nx) {
  return ((long long)y * nx + x) * P::kRest + c;
}
template <class P>
__device__ __forceinline__ long long aux_idx(int c, int y, int x, int nx) {
  return ((long long)y * nx + x) * P::kAux + c;
}

// Rows y-1, y, y+1 to pull from (valid even at walls) and the wall flags of
// row y.
struct RowN {
  int m, c, p;
  bool bot, top;
};

__device__ __forceinline__ RowN row_numbers(int y, int ny, int walls) {
  const RowIdx r = row_index(y, 1, ny, walls);
  RowN n;
  n.m = int(r.rm);
  n.c = int(r.rc);
  n.p = int(r.rp);
  n.bot = r.bot;
  n.top = r.top;
  return n;
}

// Source (row, column, direction) of population i pulled to site (x, row
// r.c): x - c_i, or across a wall the opposite population of the site
// itself (half-way bounce-back).
struct Src {
  int y, x, dir;
};
__device__ __forceinline__ Src pull_source(int i, const RowN &r, int x, int xm, int xp) {
  switch (i) {
    case 0: return {r.c, x, 0};
    case 1: return {r.c, xm, 1};
    case 3: return {r.c, xp, 3};
    case 2: return r.bot ? Src{r.c, x, 4} : Src{r.m, x, 2};
    case 5: return r.bot ? Src{r.c, x, 7} : Src{r.m, xm, 5};
    case 6: return r.bot ? Src{r.c, x, 8} : Src{r.m, xp, 6};
    case 4: return r.top ? Src{r.c, x, 2} : Src{r.p, x, 4};
    case 7: return r.top ? Src{r.c, x, 5} : Src{r.p, xp, 7};
    default: return r.top ? Src{r.c, x, 6} : Src{r.p, xm, 8};
  }
}

// Pull streaming of f and g to site (x, row) (pointer form, for the
// per-site kernels).
template <class P>
__device__ __forceinline__ void pull_fg(const typename P::S *__restrict__ s, const RowN &r,
                                        int x, int xm, int xp, int nx, typename P::R fi,
                                        typename P::R gi, typename P::R *f,
                                        typename P::R *g) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const Src q = pull_source(i, r, x, xm, xp);
    f[i] = ld<P>(s, fg_idx(q.dir, 0, q.y, q.x, nx), fi);
    g[i] = ld<P>(s, fg_idx(q.dir, 1, q.y, q.x, nx), gi);
  }
}

// Pull of h_1..h_8 (h[k] = h_{k+1}); across a wall, bounce-back with Ladd's
// moving-wall term 2 w_i rho_w (c_i.u_w)/c_s^2 = rho_w c_ix u_w / 6 for the
// diagonal populations (rho_w = rho at the site at collision time).
template <class P>
__device__ __forceinline__ void pull_h(const typename P::S *__restrict__ s, const RowN &r,
                                       int x, int xm, int xp, int nx, typename P::R inv,
                                       typename P::R rho_w, typename P::R uwb,
                                       typename P::R uwt, typename P::R *h) {
  using R = typename P::R;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const Src q = pull_source(i, r, x, xm, xp);
    h[i - 1] = ld<P>(s, h_idx(q.dir, q.y, q.x, nx), inv);
  }
  const R kb = rho_w * uwb * R(1.0 / 6.0), kt = rho_w * uwt * R(1.0 / 6.0);
  if (r.bot) {
    h[4] += kb;
    h[5] -= kb;
  }
  if (r.top) {
    h[6] -= kt;
    h[7] += kt;
  }
}

// Rest values of the nine source sites of a row r relative to the site's
// own value: e_i = X(x - c_i) - X(x); bounced populations come from the
// site itself (e_i = 0).  v holds X at rows r-1 (m), r (c), r+1 (n) of
// columns x-1 (L), x, x+1 (R).
// Rest part of h_k under float16 storage: 3 w_k (P + c_k . j), j = rho u,
// with (sx, sy) = c_k.  The storing site subtracts it for each outgoing k
// and the receiving site adds the same expression of the same stored
// values back, so the two cancel exactly.
template <class R>
__device__ __forceinline__ R hb(R w3, R P, int sx, R jx, int sy, R jy) {
#pragma clang fp contract(off)
  R t = P;
  if (sx > 0) t += jx;
  if (sx < 0) t -= jx;
  if (sy > 0) t += jy;
  if (sy < 0) t -= jy;
  return w3 * t;
}
template <class R>
struct HRest {
  R P, jx, jy;
};
// Rest parts of the post-collision h_1..h_8 stored at one site (b[k] for
// h_{k+1}).
template <class R>
__device__ __forceinline__ void h_store_basis(const HRest<R> &v, R *b) {
#pragma clang fp contract(off)
  const R a = R(1) / R(3), d = R(1) / R(12);  // 3 w_k
  b[0] = hb(a, v.P, 1, v.jx, 0, v.jy);
  b[1] = hb(a, v.P, 0, v.jx, 1, v.jy);
  b[2] = hb(a, v.P, -1, v.jx, 0, v.jy);
  b[3] = hb(a, v.P, 0, v.jx, -1, v.jy);
  b[4] = hb(d, v.P, 1, v.jx, 1, v.jy);
  b[5] = hb(d, v.P, -1, v.jx, 1, v.jy);
  b[6] = hb(d, v.P, -1, v.jx, -1, v.jy);
  b[7] = hb(d, v.P, 1, v.jx, -1, v.jy);
}
// Rest parts of the h_1..h_8 arriving at a site from the 9-point windows
// of the stored (P, jx, jy): each from its source site x - c_k, or at a
// wall row from the site itself, where the arriving h_k left as h_-k.
template <class R>
__device__ __forceinline__ void h_arrival_basis(const Nine<R> &P, const Nine<R> &jx,
                                                const Nine<R> &jy, bool bot, bool top, R *b) {
#pragma clang fp contract(off)
  const R a = R(1) / R(3), d = R(1) / R(12);
  b[0] = hb(a, P.cL, 1, jx.cL, 0, jy.cL);
  b[2] = hb(a, P.cR, -1, jx.cR, 0, jy.cR);
  b[1] = bot ? hb(a, P.c, 0, jx.c, -1, jy.c) : hb(a, P.m, 0, jx.m, 1, jy.m);
  b[4] = bot ? hb(d, P.c, -1, jx.c, -1, jy.c) : hb(d, P.mL, 1, jx.mL, 1, jy.mL);
  b[5] = bot ? hb(d, P.c, 1, jx.c, -1, jy.c) : hb(d, P.mR, -1, jx.mR, 1, jy.mR);
  b[3] = top ? hb(a, P.c, 0, jx.c, 1, jy.c) : hb(a, P.n, 0, jx.n, -1, jy.n);
  b[6] = top ? hb(d, P.c, 1, jx.c, 1, jy.c) : hb(d, P.nR, -1, jx.nR, -1, jy.nR);
  b[7] = top ? hb(d, P.c, -1, jx.c, 1, jy.c) : hb(d, P.nL, 1, jx.nL, -1, jy.nL);
}

template <class R>
__device__ __forceinline__ void source_offsets(const Nine<R> &v, bool bot, bool top, R *e) {
  const R c = v.c;
  e[0] = R(0);
  e[1] = v.cL - c;
  e[3] = v.cR - c;
  e[2] = bot ? R(0) : v.m - c;
  e[5] = bot ? R(0) : v.mL - c;
  e[6] = bot ? R(0) : v.mR - c;
  e[4] = top ? R(0) : v.n - c;
  e[7] = top ? R(0) : v.nR - c;
  e[8] = top ? R(0) : v.nL - c;
}

// Value of lane-1 / lane+1 of the wavefront: DPP wave shifts (one VALU op
// per 32 bits; lane 0 / lane 63 receive 0, which is never used).
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_left(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0x138, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x138, 0xf, 0xf, true);
  return __longlong_as_double((long long)((unsigned long long)(unsigned)lo |
                                          ((unsigned long long)(unsigned)hi << 32)));
}
__device__ __forceinline__ double from_right(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0x130, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x130, 0xf, 0xf, true);
  return __longlong_as_double((long long)((unsigned long long)(unsigned)lo |
                                          ((unsigned long long)(unsigned)hi << 32)));
}

// 3x3 neighbourhood of site k of a lane that holds K adjacent columns,
// from the lane's values in rows y-1 (m), y (c), y+1 (n): neighbours
// across the lane's edge come from the adjacent lanes.
template <int K, int k, class R>
__device__ __forceinline__ Nine<R> window_k(const R *m, const R *c, const R *n) {
  Nine<R> v;
  v.m = m[k];
  v.c = c[k];
  v.n = n[k];
  if constexpr (k > 0) {
    v.mL = m[k - 1];
    v.cL = c[k - 1];
    v.nL = n[k - 1];
  } else {
    v.mL = from_left(m[K - 1]);
    v.cL = from_left(c[K - 1]);
    v.nL = from_left(n[K - 1]);
  }
  if constexpr (k < K - 1) {
    v.mR = m[k + 1];
    v.cR = c[k + 1];
    v.nR = n[k + 1];
  } else {
    v.mR = from_right(m[0]);
    v.cR = from_right(c[0]);
    v.nR = from_right(n[0]);
  }
  return v;
}

// Values of K adjacent columns pulled by one column to the right (sh = 1:
// site k takes column k-1, site 0 the last column of the lane to the
// left), to the left (sh = -1), or not at all (sh = 0).  sh is
// wavefront-uniform; at wall rows the bounced populations are not shifted.
template <int K, class R>
__device__ __forceinline__ void shift_k(const R *v, int sh, R *out) {
  R l[K], r[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    l[k] = k > 0 ? v[k > 0 ? k - 1 : 0] : from_left(v[K - 1]);
    r[k] = k < K - 1 ? v[k < K - 1 ? k + 1 : 0] : from_right(v[0]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) out[k] = sh > 0 ? l[k] : (sh < 0 ? r[k] : v[k]);
}


// Pairs through one buffer access.  Vector elements are copied to scalars
// before any reinterpretation: a bit cast applied directly to an element
// of an ext_vector reads the vector's first element.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <class T>
struct PairIO;
template <>
struct PairIO<float> {
  static __device__ __forceinline__ void load(rsrc_t r, unsigned v, unsigned s, float &a,
                                              float &b) {
    const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0);
    const unsigned w0 = w[0], w1 = w[1];
    a = __uint_as_float(w0);
    b = __uint_as_float(w1);
  }
  template <int POL>
  static __device__ __forceinline__ void store(float a, float b, rsrc_t r, unsigned v,
                                               unsigned s) {
    u32x2 w;
    w[0] = __float_as_uint(a);
    w[1] = __float_as_uint(b);
    __builtin_amdgcn_raw_buffer_store_b64(w, r, v, s, POL);
  }
};
template <>
struct PairIO<double> {
  static __device__ __forceinline__ void load(rsrc_t r, unsigned v, unsigned s, double &a,
                                              double &b) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, v, s, 0);
    const unsigned w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
    a = __hiloint2double(int(w1), int(w0));
    b = __hiloint2double(int(w3), int(w2));
  }
  template <int POL>
  static __device__ __forceinline__ void store(double a, double b, rsrc_t r, unsigned v,
                                               unsigned s) {
    u32x4 w;
    w[0] = unsigned(__double2loint(a));
    w[1] = unsigned(__double2hiint(a));
    w[2] = unsigned(__double2loint(b));
    w[3] = unsigned(__double2hiint(b));
    wide_store_begin();
    __builtin_amdgcn_raw_buffer_store_b128(w, r, v, s, POL);
    wide_store_guard();
  }
};
template <>
struct PairIO<_Float16> {
  static __device__ __forceinline__ void load(rsrc_t r, unsigned v, unsigned s, _Float16 &a,
                                              _Float16 &b) {
    const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0);
    const unsigned short lo = (unsigned short)(w & 0xffffu), hi = (unsigned short)(w >> 16);
    a = __builtin_bit_cast(_Float16, lo);
    b = __builtin_bit_cast(_Float16, hi);
  }
};

// Three floats through one 96-bit load.
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
struct TripleIO {
  static __device__ __forceinline__ void load(rsrc_t r, unsigned v, unsigned s, float &a,
                                              float &b, float &c) {
    const u32x3 w = __builtin_amdgcn_raw_buffer_load_b96(r, v, s, 0);
    const unsigned w0 = w[0], w1 = w[1], w2 = w[2];
    a = __uint_as_float(w0);
    b = __uint_as_float(w1);
    c = __uint_as_float(w2);
  }
};

// Four floats through one 128-bit access.
struct QuadIO {
  static __device__ __forceinline__ void load(rsrc_t r, unsigned v, unsigned s, float &a,
                                              float &b, float &c, float &d) {
    const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(r, v, s, 0);
    const unsigned w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
    a = __uint_as_float(w0);
    b = __uint_as_float(w1);
    c = __uint_as_float(w2);
    d = __uint_as_float(w3);
  }
  template <int POL>
  static __device__ __forceinline__ void store(float a, float b, float c, float d, rsrc_t r,
                                               unsigned v, unsigned s) {
    u32x4 w;
    w[0] = __float_as_uint(a);
    w[1] = __float_as_uint(b);
    w[2] = __float_as_uint(c);
    w[3] = __float_as_uint(d);
    wide_store_begin();
    __builtin_amdgcn_raw_buffer_store_b128(w, r, v, s, POL);
    wide_store_guard();
  }
};

// The row number as the loop's optimiser cannot follow it (readfirstlane
// of a wave-uniform value: the same number).  The row loop passes each
// row through it, so the byte offsets derived from the row (one per
// population plane and record) are computed where they are used, by scalar
// adds, instead of each becoming an induction variable of its own: those
// outnumbered the scalar registers, and the excess was kept in vector lanes
// at one v_readlane per use (float32 step: 28 such registers, none now;
// 1.5% faster on the 2048x2048 field).
__device__ __forceinline__ int opaque_row(int y) {
  return __builtin_amdgcn_readfirstlane(y);
}

// Byte offsets of one row in the step kernel's three groups.
struct RowOff {
  unsigned m, c, p;  // population rows y-1, y, y+1
  bool bot, top;
};

__device__ __forceinline__ RowOff row_offsets(int y, int ny, int walls, unsigned row_bytes) {
  const RowIdx r = row_index(y, 1, ny, walls);
  RowOff o;
  o.m = unsigned(r.rm) * row_bytes;
  o.c = unsigned(r.rc) * row_bytes;
  o.p = unsigned(r.rp) * row_bytes;
  o.bot = r.bot;
  o.top = r.top;
  return o;
}

// Per-lane byte offsets of columns x, x-1, x+1 inside a FG block (pairs)
// and an H block (singles).
struct ColOff {
  unsigned p0, pm, pp;  // pairs
  unsigned h0, hm, hp;  // singles
};

template <class P>
struct Pull {
  using R = typename P::R;
  using S = typename P::S;
  // f_i, g_i of the nine populations arriving at row r (one pair load each)
  static __device__ __forceinline__ void fg(rsrc_t rs, unsigned nxb, const RowOff &r,
                                            const ColOff &c, const Scales<P> &sc, R *f, R *g) {
    // nxb: bytes of one pair row (nx pairs)
    auto pair = [&](int dir, unsigned row, unsigned col, int i) {
#pragma clang fp contract(off)
      S a, b;
      PairIO<S>::load(rs, col, row + unsigned(dir) * nxb, a, b);
      if constexpr (P::SCALED) {
        f[i] = R(a) * sc.fi;
        g[i] = R(b) * sc.gi;
      } else {
        f[i] = R(a);
        g[i] = R(b);
      }
    };
    // One load per population on every path: at a wall row the source of
    // the three populations leaving through the wall is selected (uniform
    // over the wavefront), not branched to, so every row issues the same
    // sequence of memory operations.
    const bool bot = r.bot, top = r.top;
    pair(0, r.c, c.p0, 0);
    pair(1, r.c, c.pm, 1);
    pair(3, r.c, c.pp, 3);
    pair(0, bot ? r.c + 4 * nxb : r.m + 2 * nxb, c.p0, 2);
    pair(0, bot ? r.c + 7 * nxb : r.m + 5 * nxb, bot ? c.p0 : c.pm, 5);
    pair(0, bot ? r.c + 8 * nxb : r.m + 6 * nxb, bot ? c.p0 : c.pp, 6);
    pair(0, top ? r.c + 2 * nxb : r.p + 4 * nxb, c.p0, 4);
    pair(0, top ? r.c + 5 * nxb : r.p + 7 * nxb, top ? c.p0 : c.pp, 7);
    pair(0, top ? r.c + 6 * nxb : r.p + 8 * nxb, top ? c.p0 : c.pm, 8);
  }
  // h_1..h_8 arriving at row r (h[k] = h_{k+1}); hb: byte offset of the H
  // block in a row, nxh: bytes of one h row
  static __device__ __forceinline__ void h(rsrc_t rs, unsigned hb, unsigned nxh,
                                           const RowOff &r, const ColOff &c, R inv, R *out) {
    // off: byte offset of the source row and direction plane within the
    // H block; wall rows select their bounced source as in fg()
    auto one = [&](unsigned off, unsigned col, int k) {
      out[k] = bld<P>(rs, col, off + hb, inv);
    };
    const bool bot = r.bot, top = r.top;
    one(r.c, c.hm, 0);             // h_1 from x-1
    one(r.c + 2 * nxh, c.hp, 2);   // h_3 from x+1
    one(bot ? r.c + 3 * nxh : r.m + nxh, c.h0, 1);                    // h_2
    one(bot ? r.c + 6 * nxh : r.m + 4 * nxh, bot ? c.h0 : c.hm, 4);   // h_5
    one(bot ? r.c + 7 * nxh : r.m + 5 * nxh, bot ? c.h0 : c.hp, 5);   // h_6
    one(top ? r.c + nxh : r.p + 3 * nxh, c.h0, 3);                    // h_4
    one(top ? r.c + 4 * nxh : r.p + 6 * nxh, top ? c.h0 : c.hp, 6);   // h_7
    one(top ? r.c + 5 * nxh : r.p + 7 * nxh, top ? c.h0 : c.hm, 7);   // h_8
  }
};

// Moving-wall term of the bounced diagonal h populations (see pull_h).
template <class R>
__device__ __forceinline__ void wall_terms(bool bot, bool top, R rho_w, R uwb, R uwt,
                                           R *h) {
  if (bot) {
    const R kb = rho_w * uwb * R(1.0 / 6.0);
    h[4] += kb;
    h[5] -= kb;
  }
  if (top) {
    const R kt = rho_w * uwt * R(1.0 / 6.0);
    h[6] -= kt;
    h[7] += kt;
  }
}

// Strip geometry of the step kernel with K adjacent columns per lane: two
// halo columns on each side (2 / K lanes), the rest interior.
template <int K>
struct Strip {
  static constexpr int kHaloLanes = 2 / K;
  static constexpr int kCols = K * (kWave - 2 * kHaloLanes);  // interior columns
};

// s_waitcnt operand (gfx9 encoding) that waits for all vector memory
// operations only: vmcnt 0, expcnt and lgkmcnt at their maxima.
constexpr int kWaitVmcnt0 = (0xF << 8) | (0x7 << 4);

template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

// f(std::integral_constant<int, k>) for k = 0 .. N-1, unrolled.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Float16 halves of a 32-bit word.
__device__ __forceinline__ float half_lo(unsigned w) {
  return float(__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu)));
}
__device__ __forceinline__ float half_hi(unsigned w) {
  return float(__builtin_bit_cast(_Float16, (unsigned short)(w >> 16)));
}
// A widened float16 value times a scale, rounded once: written as a fused
// multiply-add with +0 so that the widening and the product are one
// mixed-precision instruction (v_fma_mix_f32).  The result is the rounded
// product, except that a product of -0 becomes +0.
__device__ __forceinline__ float scale_half(float h, float s) { return __builtin_fmaf(h, s, 0.0f); }
__device__ __forceinline__ unsigned halves(float lo, float hi) {
  const unsigned short a = __builtin_bit_cast(unsigned short, _Float16(lo)),
                       b = __builtin_bit_cast(unsigned short, _Float16(hi));
  return unsigned(a) | (unsigned(b) << 16);
}

// Float16 storage rounds stochastically.  Round-to-nearest of a slowly
// varying value makes nearly the same error every step, and those errors
// add up linearly in time; stochastic rounding makes them unbiased and
// uncorrelated.  Measured on the 100x100 convection test (u = 0.05, 2000
// steps) the phi error against float64 falls from 4.2e-3 to 1.3e-4.
//
// Integer hash (multiply-xorshift; the constants of C. Wellons' lowbias32).
__device__ __forceinline__ unsigned hash32(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
// Two values to packed float16, rounded stochastically: 13 bits of a hash
// of both values' float32 bits and of key are added below the 10 kept
// mantissa bits, and the sum is truncated (round toward zero), so a value
// rounds away from zero with probability equal to its fractional distance.
// The bits come from the values themselves, so the rounding is reproducible
// and changes from step to step as the values do.  (Below the smallest
// normal float16, 2^-14, more than 13 bits are dropped and the rounding
// leans toward zero: at the default scales that is below 1.5e-8 of f and g
// and 1e-9 of h.)
__device__ __forceinline__ unsigned halves_sr(float lo, float hi, unsigned key) {
  const unsigned bl = __float_as_uint(lo), bh = __float_as_uint(hi);
  const unsigned r = hash32(bl ^ ((bh << 16) | (bh >> 16)) ^ key);
  const float a = __uint_as_float(bl + (r & 0x1fffu));
  const float b = __uint_as_float(bh + ((r >> 16) & 0x1fffu));
  return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(a, b));
}
// Packed float16 words (f_i, g_i) of one site's nine scaled deviations:
// i = 1..8 rounded stochastically; their rounding errors (exact in float32)
// are added to the rest population, which stays at the site and is rounded
// to nearest.  The deviations of a site sum to zero, so the stored ones
// change the mass by that one rounding only, not by nine random ones.
// amax takes the largest magnitude packed: the conversion saturates at the
// float16 maximum 65504 without a sign of it, so the caller flags larger
// values (or NaN) as a lost state.
__device__ __forceinline__ void pack_fg(const float *f, const float *g, float sf, float sg,
                                        unsigned site, unsigned *w, float &amax) {
#pragma clang fp contract(off)
  float ef = -0.f, eg = -0.f;  // -0 + x is x: the first sum needs no add
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const float vf = f[i] * sf, vg = g[i] * sg;
    amax = fmaxf(amax, fmaxf(fabsf(vf), fabsf(vg)));
    w[i] = halves_sr(vf, vg, site * 32u + unsigned(i));
    ef += vf - half_lo(w[i]);
    eg += vg - half_hi(w[i]);
  }
  const float v0 = f[0] * sf + ef, u0 = g[0] * sg + eg;
  amax = fmaxf(amax, fmaxf(fabsf(v0), fabsf(u0)));
  w[0] = halves(v0, u0);
}
constexpr float kHalfMax = 65504.f;  // largest finite float16

// Pull streaming with two adjacent columns per lane (float32 storage, or
// scaled float16 deviations): each population is loaded at the lane's own
// two columns, one (f, g) access (16 bytes float32, 8 bytes float16) and
// one h access (8 or 4 bytes) per plane; sources, bounce-back selection
// and load order as in Pull.  The shift by c_ix is applied in registers by
// shift_fg / shift_h when the row is used, not at the load, so the loads
// of the next row stay in flight meanwhile.  Float16 words are kept packed
// until then (decode_fg / decode_h): the prefetched row then holds half the
// registers, and no conversion consumes a load early.
template <class P>
struct Pull2 {
  using R = typename P::R;
  using S = typename P::S;
  static_assert((!P::SCALED && sizeof(S) == 4) || (P::SCALED && sizeof(S) == 2),
                "float32 or scaled float16 storage");
  static __device__ __forceinline__ void fg(rsrc_t rs, unsigned nxb, const RowOff &r,
                                            unsigned col, R (*f)[9], R (*g)[9]) {
    auto quad = [&](unsigned row, int i) {
      if constexpr (sizeof(S) == 4) {
        QuadIO::load(rs, col, row, f[0][i], g[0][i], f[1][i], g[1][i]);
      } else {  // packed (f, g) words of the two columns, decoded in decode_fg
        const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, col, row, 0);
        const unsigned w0 = w[0], w1 = w[1];
        f[0][i] = __uint_as_float(w0);
        f[1][i] = __uint_as_float(w1);
        g[0][i] = g[1][i] = R(0);
      }
    };
    const bool bot = r.bot, top = r.top;
    quad(r.c, 0);
    quad(r.c + nxb, 1);
    quad(r.c + 3 * nxb, 3);
    quad(bot ? r.c + 4 * nxb : r.m + 2 * nxb, 2);
    quad(bot ? r.c + 7 * nxb : r.m + 5 * nxb, 5);
    quad(bot ? r.c + 8 * nxb : r.m + 6 * nxb, 6);
    quad(top ? r.c + 2 * nxb : r.p + 4 * nxb, 4);
    quad(top ? r.c + 5 * nxb : r.p + 7 * nxb, 7);
    quad(top ? r.c + 6 * nxb : r.p + 8 * nxb, 8);
  }
  // float16 storage: unpack and scale what fg() loaded.  The scaled values
  // are rounded here (no contraction into the sums that use them), so the
  // result does not depend on which copy of the row code a site runs in.
  static __device__ __forceinline__ void decode_fg(const Scales<P> &sc, R (*f)[9], R (*g)[9]) {
    if constexpr (sizeof(S) == 2) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const unsigned w0 = __float_as_uint(f[0][i]), w1 = __float_as_uint(f[1][i]);
        f[0][i] = scale_half(half_lo(w0), sc.fi);
        g[0][i] = scale_half(half_hi(w0), sc.gi);
        f[1][i] = scale_half(half_lo(w1), sc.fi);
        g[1][i] = scale_half(half_hi(w1), sc.gi);
      }
    }
  }
  // float16 storage: unpack and scale what h() loaded
  static __device__ __forceinline__ void decode_h(R inv, R (*h)[8]) {
    if constexpr (sizeof(S) == 2) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const unsigned w = __float_as_uint(h[0][k]);
        h[0][k] = scale_half(half_lo(w), inv);
        h[1][k] = scale_half(half_hi(w), inv);
      }
    }
  }
  // shift of population i (1: from the left column, -1: from the right);
  // populations bounced at a wall row come from the site itself
  static __device__ __forceinline__ int shift_of(int i, bool bot, bool top) {
    switch (i) {
      case 1: return 1;
      case 3: return -1;
      case 5: return bot ? 0 : 1;
      case 6: return bot ? 0 : -1;
      case 7: return top ? 0 : -1;
      case 8: return top ? 0 : 1;
      default: return 0;
    }
  }
  static __device__ __forceinline__ void shift_fg(bool bot, bool top, R (*f)[9], R (*g)[9]) {
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int sh = shift_of(i, bot, top);
      if (i == 2 || i == 4) continue;
      R a[2] = {f[0][i], f[1][i]}, b[2] = {g[0][i], g[1][i]}, oa[2], ob[2];
      shift_k<2>(a, sh, oa);
      shift_k<2>(b, sh, ob);
      f[0][i] = oa[0];
      f[1][i] = oa[1];
      g[0][i] = ob[0];
      g[1][i] = ob[1];
    }
  }
  static __device__ __forceinline__ void h(rsrc_t rs, unsigned hb, unsigned nxh,
                                           const RowOff &r, unsigned col, R (*out)[8]) {
    auto two = [&](unsigned off, int k) {
      if constexpr (sizeof(S) == 4) {
        PairIO<float>::load(rs, col, off + hb, out[0][k], out[1][k]);
      } else {  // packed h word of the two columns, decoded in decode_h
        const unsigned w = __builtin_amdgcn_raw_buffer_load_b32(rs, col, off + hb, 0);
        out[0][k] = __uint_as_float(w);
        out[1][k] = R(0);
      }
    };
    const bool bot = r.bot, top = r.top;
    two(r.c, 0);                                   // h_1
    two(r.c + 2 * nxh, 2);                         // h_3
    two(bot ? r.c + 3 * nxh : r.m + nxh, 1);       // h_2
    two(bot ? r.c + 6 * nxh : r.m + 4 * nxh, 4);   // h_5
    two(bot ? r.c + 7 * nxh : r.m + 5 * nxh, 5);   // h_6
    two(top ? r.c + nxh : r.p + 3 * nxh, 3);       // h_4
    two(top ? r.c + 4 * nxh : r.p + 6 * nxh, 6);   // h_7
    two(top ? r.c + 5 * nxh : r.p + 7 * nxh, 7);   // h_8
  }
  // h[k] = h_{k+1}
  static __device__ __forceinline__ void shift_h(bool bot, bool top, R (*h)[8]) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k == 1 || k == 3) continue;
      const int sh = shift_of(k + 1, bot, top);
      R a[2] = {h[0][k], h[1][k]}, o[2];
      shift_k<2>(a, sh, o);
      h[0][k] = o[0];
      h[1][k] = o[1];
    }
  }
};

// The fused step: pull-stream + boundaries, phi/psi/sigma, stencils, forces,
// closures, three MRT collisions, store.  Each lane holds K adjacent
// columns.  The two columns on each side of the interior are halo: they
// rebuild phi, psi, sigma for the stencils of the interior columns but
// store nothing (the outermost one only serves the rebuild of the next,
// which needs the old rest values one column further out).
// The row loop is software-pipelined: the loads for row y+1 are issued
// before the arithmetic and stores of row y.
// One tile (strip x rows) of one simulation, executed by one wavefront.
// NS: velocity from the Navier-Stokes LB (h); otherwise prescribed (u held
// in aux slots 0, 1; only f and g evolve).
// K = 2 (float32 storage, even nx): every access of a lane covers two
// sites, 16 bytes per (f, g) plane and 8 per h plane.
template <class P, int K, bool GENR, bool HAS_S, bool NS>
__device__ __forceinline__ void step_tile(const StepArgs<P> &a, const int strip, const int y0,
                                          const int y1) {
  using R = typename P::R;
  using S = typename P::S;
  using A = typename P::A;
  static_assert(K == 1 || (K == 2 && sizeof(A) == 4 &&
                           ((!P::SCALED && sizeof(S) == 4) || (P::SCALED && sizeof(S) == 2))),
                "two columns per lane: float32 or float16 storage");
  constexpr int HL = Strip<K>::kHaloLanes;
  constexpr int COLS = Strip<K>::kCols;
  const int lane = threadIdx.x & (kWave - 1);
  const int nx = a.nx, ny = a.ny, walls = a.walls;
  const int x0 = strip * COLS;
  const int wl = min(COLS, nx - x0) / K;  // interior lanes (nx is a multiple of K)
  const bool interior = lane >= HL && lane < HL + wl;
  int xl = x0 - K * HL + K * min(lane, wl + 2 * HL - 1);  // first column of the lane
  xl %= nx;
  if (xl < 0) xl += nx;
  const unsigned xc = unsigned(xl);
  const unsigned xcm = xl == 0 ? unsigned(nx - 1) : xc - 1;
  const unsigned xcp = xl == nx - 1 ? 0u : xc + 1;
  constexpr unsigned ES = sizeof(S), EA = sizeof(A);
  ColOff co;
  co.p0 = xc * 2 * ES;
  co.pm = xcm * 2 * ES;
  co.pp = xcp * 2 * ES;
  co.h0 = xc * ES;
  co.hm = xcm * ES;
  co.hp = xcp * ES;
  const unsigned brest = xc * P::kRest * EA;  // this lane's first rest record in a row
  const unsigned baux = xc * P::kAux * EA;    // this lane's first aux record
  const unsigned nsites = unsigned(nx) * unsigned(ny);
  const unsigned nxb = unsigned(nx) * 2 * ES;      // one FG pair row
  const unsigned nxh = unsigned(nx) * ES;          // one h row
  const unsigned hb = 9u * nxb;                    // H block offset in a row
  const unsigned rows_s = unsigned(kPlanes) * nxh; // bytes per population row
  const unsigned rrow = unsigned(nx) * P::kRest * EA; // bytes per rest row
  const unsigned arow = unsigned(nx) * P::kAux * EA;  // bytes per aux row
  const rsrc_t rsrc = make_rsrc(a.src, unsigned(kPlanes) * nsites * ES);
  const rsrc_t rdst = make_rsrc(a.dst, unsigned(kPlanes) * nsites * ES);
  const rsrc_t rrest = make_rsrc(a.src_rest, unsigned(P::kRest) * nsites * EA);
  const rsrc_t rdrest = make_rsrc(a.dst_rest, unsigned(P::kRest) * nsites * EA);
  const rsrc_t raux = make_rsrc(a.aux, unsigned(P::kAux) * nsites * EA);
  const Phys<R> &p = a.p;
  const Scales<P> &sc = a.sc;
  // the aux records (ux, uy) of a lane's two float32 sites: one 16-byte access
  constexpr bool kAuxQuad = sizeof(A) == 4 && K == 2;
  // the step reads an aux record: the previous velocity, or the prescribed one
  constexpr bool kAuxRead = !P::HDEV || !NS;

  // old (phi, psi) of this lane's columns at row y, wrapped or clamped
  auto rest_at = [&](int y, R *X, R *Y) {
    const unsigned ro = unsigned(wrap_row(y, ny, walls)) * rrow;
    if constexpr (K == 2 && P::kRest == 2) {  // both records in one access
      QuadIO::load(rrest, brest, ro, X[0], Y[0], X[1], Y[1]);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        A u, v;
        PairIO<A>::load(rrest, brest + unsigned(k) * P::kRest * EA, ro, u, v);
        X[k] = R(u);
        Y[k] = R(v);
      }
    }
  };
  // raw stored deviations of f and g pulled to row r
  auto load_fg = [&](int r, R (*d)[9], R (*q)[9]) {
    const RowOff o = row_offsets(r, ny, walls, rows_s);
    if constexpr (K == 1)
      Pull<P>::fg(rsrc, nxb, o, co, sc, d[0], q[0]);
    else
      Pull2<P>::fg(rsrc, nxb, o, co.p0, d, q);
  };
  // loads of row y that the rebuild of row y+1 does not need
  auto load_row = [&](int y, R (*h)[8], R *uxp, R *uyp) {
    if constexpr (NS) {
      const RowOff o = row_offsets(y, ny, walls, rows_s);
      if constexpr (K == 1)
        Pull<P>::h(rsrc, hb, nxh, o, co, sc.hi, h[0]);
      else
        Pull2<P>::h(rsrc, hb, nxh, o, co.h0, h);
    }
    // u: the previous level, or the prescribed field; with float16 storage
    // the previous velocity comes from the rest record (P, rho u) instead
    if constexpr (!kAuxRead) {
#pragma unroll
      for (int k = 0; k < K; ++k) uxp[k] = uyp[k] = R(0);
    } else if constexpr (kAuxQuad) {  // (ux, uy) of both sites in one access
      QuadIO::load(raux, baux, unsigned(y) * arow, uxp[0], uyp[0], uxp[1], uyp[1]);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        A u, v;
        PairIO<A>::load(raux, baux + unsigned(k) * P::kAux * EA, unsigned(y) * arow, u, v);
        uxp[k] = R(u);
        uyp[k] = R(v);
      }
    }
  };
  // old (P, rho ux, rho uy) of this lane's columns at row y (float16
  // storage only)
  struct HR {
    R pr[K], jx[K], jy[K];
  };
  auto hrest_at = [&](int y, HR &v) {
    if constexpr (P::HDEV && NS) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        TripleIO::load(rrest, brest + unsigned(k) * P::kRest * EA + 2 * EA,
                       unsigned(wrap_row(y, ny, walls)) * rrow, v.pr[k], v.jx[k], v.jy[k]);
    }
  };
  // rebuild row r from its raw deviations: new phi, psi, sigma, and the
  // deviations relative to them (in place), given the old rest fields at
  // rows r-1, r, r+1 of the lane's columns
  auto rebuild = [&](int r, const R *Xm, const R *Xc, const R *Xn, const R *Ym, const R *Yc,
                     const R *Yn, R (*d)[9], R (*q)[9], R *ph, R *ps, R *sg) {
    const bool bot = walls && r == 0, top = walls && r == ny - 1;
    if constexpr (K == 2) {
      Pull2<P>::decode_fg(sc, d, q);
      Pull2<P>::shift_fg(bot, top, d, q);
    }
    static_for<K>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      R e[9];
      source_offsets(window_k<K, k>(Xm, Xc, Xn), bot, top, e);
      ph[k] = restream(d[k], e, Xc[k]);
      source_offsets(window_k<K, k>(Ym, Yc, Yn), bot, top, e);
      ps[k] = restream(q[k], e, Yc[k]);
      sg[k] = sigma_of(p, ps[k]);
    });
  };
  auto copy = [](R *dst, const R *src) {
#pragma unroll
    for (int k = 0; k < K; ++k) dst[k] = src[k];
  };

  // Prologue: phi, psi, sigma of rows y0 and y0-1, and the loop's first
  // prefetch.  With float32 and float64 storage every load is issued before
  // the first rebuild, so a tile starts after one round trip to memory
  // rather than three (1% faster on the 2048x2048 field for float64, 4-10%
  // shorter steps on grids too small to fill the device).  Float16 storage
  // keeps the rebuilds between the loads (3% faster there).
  constexpr bool kEarlyLoads = !P::SCALED;
  // old rest values of this lane's columns, rows y-1 .. y+2
  R X0[K], X1[K], X2[K], X3[K], Y0[K], Y1[K], Y2[K], Y3[K];
  rest_at(y0 - 1, X0, Y0);
  rest_at(y0, X1, Y1);
  rest_at(y0 + 1, X2, Y2);
  rest_at(y0 + 2, X3, Y3);
  R dc[K][9], qc[K][9];
  R phc[K], psc[K], sgc[K], phm[K], psm[K], sgm[K];
  load_fg(y0, dc, qc);
  // row y0-1, unless it is the mirror ghost below the bottom wall
  const bool ghost_below = walls && y0 == 0;
  const int ym = y0 == 0 ? ny - 1 : y0 - 1;
  R dt[K][9], qt[K][9], Xa[K], Ya[K];
  auto load_below = [&]() {
    if (!ghost_below) {
      rest_at(y0 - 2, Xa, Ya);
      load_fg(ym, dt, qt);
    }
  };
  auto rebuild_y0 = [&]() { rebuild(y0, X0, X1, X2, Y0, Y1, Y2, dc, qc, phc, psc, sgc); };
  auto rebuild_below = [&]() {
    if (ghost_below) {
      copy(phm, phc);
      copy(psm, psc);
      copy(sgm, sgc);
    } else {
      rebuild(ym, Xa, X0, X1, Ya, Y0, Y1, dt, qt, phm, psm, sgm);
    }
  };
  if (kEarlyLoads) {
    load_below();
  } else {
    rebuild_y0();
    load_below();
    rebuild_below();
  }

  // Software pipeline: the loads for row y+1 are issued before the
  // arithmetic and stores of row y.  Every iteration issues the same
  // memory operations on every path (no divergent or row-dependent branch
  // around a load or store), so the wait at the top of an iteration only
  // covers the loads it needs, not the stores just issued.
  R dn[K][9], qn[K][9];  // raw deviations of row y+1
  R hr[K][8];            // h of row y
  R uxr[K], uyr[K];
  // above the top wall the next row is the mirror ghost: the load of row
  // ny-1 keeps the sequence uniform and its values are not used
  auto next_fg_row = [&](int y) { return wrap_row(y, ny, walls); };
  load_fg(next_fg_row(y0 + 1), dn, qn);
  load_row(y0, hr, uxr, uyr);
  // rest (P, rho u) of rows y-1, y, y+1 and the prefetched y+2
  HR Hm{}, Hc{}, Hn{}, Hq{};
  if constexpr (P::HDEV && NS) {
    hrest_at(y0 - 1, Hm);
    hrest_at(y0, Hc);
    hrest_at(y0 + 1, Hn);
  }

  if (kEarlyLoads) {
    rebuild_y0();
    rebuild_below();
  }

  // Stores are issued by every lane (the same memory operations on every
  // path); a halo lane's offsets are kDropped, so the hardware discards its
  // part and only interior lanes write.
  const ColOff cs = {interior ? co.p0 : kDropped, 0u, 0u, interior ? co.h0 : kDropped, 0u, 0u};
  const unsigned brest_s = interior ? brest : kDropped, baux_s = interior ? baux : kDropped;
  bool bad = false;

  auto row_step = [&](int y, auto prefetch) {
    // rebuild the next row from the raw deviations loaded last iteration
    R phn[K], psn[K], sgn[K];
    const bool ghost = walls && y == ny - 1;
    if (!ghost) {
      rebuild(y + 1 == ny ? 0 : y + 1, X1, X2, X3, Y1, Y2, Y3, dn, qn, phn, psn, sgn);
    } else {  // mirror ghost row above the top wall
      copy(phn, phc);
      copy(psn, psc);
      copy(sgn, sgc);
    }
    R h[K][8];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < 8; ++i) h[k][i] = hr[k][i];
    if constexpr (K == 2 && NS) {
      Pull2<P>::decode_h(sc.hi, h);
      Pull2<P>::shift_h(walls && y == 0, walls && y == ny - 1, h);
    }
    R uxp[K], uyp[K], Sxp[K], Syp[K];
    copy(uxp, uxr);
    copy(uyp, uyr);
    // the previous level's mass flux, Eq. (16), from the previous phi of
    // rows y-1, y, y+1 (the rest values the rebuilds read)
    static_for<K>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      if constexpr (HAS_S && NS) {
        R gx, gy;
        grad9(window_k<K, k>(X0, X1, X2), gx, gy);
        mass_flux(p, X1[k], gx, gy, Sxp[k], Syp[k]);
      } else {
        Sxp[k] = Syp[k] = R(0);
      }
    });
    if constexpr (P::HDEV && NS) {  // add back the rest parts of the arriving h
      // (no contraction: float16 storage rounds stochastically from all
      // 32 bits, so every copy of the row code must give the same bits)
      static_for<K>([&](auto kc) {
#pragma clang fp contract(off)
        constexpr int k = decltype(kc)::value;
        R b[8];
        h_arrival_basis(window_k<K, k>(Hm.pr, Hc.pr, Hn.pr), window_k<K, k>(Hm.jx, Hc.jx, Hn.jx),
                        window_k<K, k>(Hm.jy, Hc.jy, Hn.jy), walls && y == 0,
                        walls && y == ny - 1, b);
#pragma unroll
        for (int i = 0; i < 8; ++i) h[k][i] += b[i];
        const R irho = recip(p.rhoB + p.drho * (X1[k] - p.phiB));
        uxp[k] = Hc.jx[k] * irho;
        uyp[k] = Hc.jy[k] * irho;
      });
    }
    R dnn[K][9], qnn[K][9];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        dnn[k][i] = dn[k][i];
        qnn[k][i] = qn[k][i];
      }

    R X4[K], Y4[K];
    copy(X4, X3);
    copy(Y4, Y3);
    if constexpr (decltype(prefetch)::value) {
      rest_at(y + 3, X4, Y4);
      load_fg(next_fg_row(y + 2), dn, qn);
      load_row(y + 1, hr, uxr, uyr);
      hrest_at(y + 2, Hq);
    }

    const bool bot = walls && y == 0, top = walls && y == ny - 1;
    R oux[K], ouy[K];
    HR hn{};
    static_for<K>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      const R php = X1[k], psp = Y1[k];
      if constexpr (NS) wall_terms(bot, top, rho_of(p, php), p.uwb, p.uwt, h[k]);

      // stencils from the register window
      const Nine<R> vphi = window_k<K, k>(phm, phc, phn);
      const Nine<R> vsig = window_k<K, k>(sgm, sgc, sgn);
      R gfx, gfy, gsx, gsy;
      grad9(vphi, gfx, gfy);
      grad9(vsig, gsx, gsy);
      const R lphi = lap9(vphi);

      Front<R> s;
      if constexpr (NS)
        site_front<R, HAS_S>(p, s, phc[k], psc[k], sgc[k], gfx, gfy, lphi, gsx, gsy, h[k], php,
                             psp, uxp[k], uyp[k], Sxp[k], Syp[k]);
      else
        site_front_prescribed<R>(p, s, phc[k], psc[k], gfx, gfy, uxp[k], uyp[k], php, psp);
      if (GENR) {
        const Nine<R> vpsi = window_k<K, k>(psm, psc, psn);
        grad9(vpsi, s.gpx, s.gpy);
      } else {
        s.gpx = s.gpy = R(0);
      }
      if constexpr (NS)
        collide_site<R, GENR>(p, s, dc[k], qc[k], h[k]);
      else
        collide_fg<R, GENR>(p, s, dc[k], qc[k]);
      if constexpr (P::HDEV && NS) {  // h as deviations from this site's new rest parts
#pragma clang fp contract(off)
        hn.pr[k] = s.P;
        hn.jx[k] = s.jx;
        hn.jy[k] = s.jy;
        R b[8];
        h_store_basis(HRest<R>{s.P, s.jx, s.jy}, b);
#pragma unroll
        for (int i = 0; i < 8; ++i) h[k][i] -= b[i];
      }
      oux[k] = s.ux;
      ouy[k] = s.uy;
      bad |= interior && !isfinite(phc[k] + psc[k] + s.ux + s.uy);
    });

    const unsigned rcs = unsigned(y) * rows_s;
    float amax = 0.f;  // largest scaled deviation stored as float16
    if constexpr (K == 1) {
      if constexpr (P::SCALED) {  // float16: packed words, stochastic rounding
        unsigned w[9];
        pack_fg(dc[0], qc[0], sc.f, sc.g, unsigned(y) * unsigned(nx) + xc, w, amax);
#pragma unroll
        for (int i = 0; i < 9; ++i)
          __builtin_amdgcn_raw_buffer_store_b32(w[i], rdst, cs.p0,
                                                rcs + unsigned(i) * nxb, P::kStorePol);
      } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
          PairIO<S>::template store<P::kStorePol>(S(dc[0][i]), S(qc[0][i]), rdst, cs.p0,
                           rcs + unsigned(i) * nxb);
      }
      if constexpr (NS && P::SCALED) {
        const unsigned key = (unsigned(y) * unsigned(nx) + xc) * 32u + 16u;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float v = h[0][i] * sc.h;
          amax = fmaxf(amax, fabsf(v));
          __builtin_amdgcn_raw_buffer_store_b16(
              (unsigned short)(halves_sr(v, 0.f, key + unsigned(i)) & 0xffffu),
              rdst, cs.h0, rcs + hb + unsigned(i) * nxh, P::kStorePol);
        }
      } else if constexpr (NS) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          bst<P>(h[0][i], rdst, cs.h0, rcs + hb + unsigned(i) * nxh);
      }
      if constexpr (P::HDEV && NS) {  // (phi, psi, P, rho ux) and rho uy
        QuadIO::store<P::kStorePol>(phc[0], psc[0], hn.pr[0], hn.jx[0], rdrest,
                                    brest_s, unsigned(y) * rrow);
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(hn.jy[0]), rdrest,
                                              brest_s + 4 * EA, unsigned(y) * rrow,
                                              P::kStorePol);
      } else {
        PairIO<A>::template store<P::kStorePol>(A(phc[0]), A(psc[0]), rdrest, brest_s,
                                                unsigned(y) * rrow);
      }
      if constexpr (!P::HDEV && NS)
        PairIO<A>::template store<P::kStorePol>(A(oux[0]), A(ouy[0]), raux, baux_s,
                                                unsigned(y) * arow);
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
      for (int i = 0; i < 9; ++i)
        QuadIO::store<P::kStorePol>(dc[0][i], qc[0][i], dc[1][i], qc[1][i], rdst,
                                    cs.p0, rcs + unsigned(i) * nxb);
      if constexpr (NS) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          PairIO<S>::template store<P::kStorePol>(
              h[0][i], h[1][i], rdst, cs.h0, rcs + hb + unsigned(i) * nxh);
      }
      QuadIO::store<P::kStorePol>(phc[0], psc[0], phc[1], psc[1], rdrest,
                                  brest_s, unsigned(y) * rrow);
      if constexpr (NS)
        QuadIO::store<P::kStorePol>(oux[0], ouy[0], oux[1], ouy[1], raux,
                                    baux_s, unsigned(y) * arow);
    } else {  // float16 deviations, scaled: four halves per (f, g) plane, two per h plane
      const unsigned site = unsigned(y) * unsigned(nx) + xc;
      unsigned w0[9], w1[9];
      pack_fg(dc[0], qc[0], sc.f, sc.g, site, w0, amax);
      pack_fg(dc[1], qc[1], sc.f, sc.g, site + 1u, w1, amax);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        u32x2 w;
        w[0] = w0[i];
        w[1] = w1[i];
        __builtin_amdgcn_raw_buffer_store_b64(w, rdst, cs.p0, rcs + unsigned(i) * nxb,
                                              P::kStorePol);
      }
      if constexpr (NS) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float v0 = h[0][i] * sc.h, v1 = h[1][i] * sc.h;
          amax = fmaxf(amax, fmaxf(fabsf(v0), fabsf(v1)));
          __builtin_amdgcn_raw_buffer_store_b32(
              halves_sr(v0, v1, site * 32u + 16u + unsigned(i)),
              rdst, cs.h0, rcs + hb + unsigned(i) * nxh, P::kStorePol);
        }
      }
      if constexpr (P::HDEV && NS) {
        // the two 5-float rest records (40 bytes) as 16 + 16 + 8 bytes
        QuadIO::store<P::kStorePol>(phc[0], psc[0], hn.pr[0], hn.jx[0], rdrest,
                                    brest_s, unsigned(y) * rrow);
        QuadIO::store<P::kStorePol>(hn.jy[0], phc[1], psc[1], hn.pr[1], rdrest,
                                    brest_s + 4 * EA, unsigned(y) * rrow);
        PairIO<A>::template store<P::kStorePol>(hn.jx[1], hn.jy[1], rdrest,
                                                brest_s + 8 * EA, unsigned(y) * rrow);
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k)
          PairIO<A>::template store<P::kStorePol>(phc[k], psc[k], rdrest,
                                                  brest_s + unsigned(k) * P::kRest * EA,
                                                  unsigned(y) * rrow);
      }
    }

    // a deviation beyond the float16 range was stored saturated: the state
    // is lost, as with a non-finite value
    if constexpr (P::SCALED) bad |= interior && !(amax <= kHalfMax);

    // slide the windows
    copy(phm, phc);
    copy(psm, psc);
    copy(sgm, sgc);
    copy(phc, phn);
    copy(psc, psn);
    copy(sgc, sgn);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        dc[k][i] = dnn[k][i];
        qc[k][i] = qnn[k][i];
      }
    copy(X0, X1);
    copy(X1, X2);
    copy(X2, X3);
    copy(X3, X4);
    copy(Y0, Y1);
    copy(Y1, Y2);
    copy(Y2, Y3);
    copy(Y3, Y4);
    if constexpr (P::HDEV && NS) {
      Hm = Hc;
      Hc = Hn;
      Hn = Hq;
    }
  };

  // The first row needs the loads just issued in any case.  Waiting for
  // them here leaves nothing of the prologue in flight at the loop head,
  // so the waits placed there serve only the previous iteration's loads
  // (long complete) instead of also holding back on its stores.
  __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
  // (This loop form, with its own trip counter and the row after the loop
  // taken from it, and the wall and wrap tests written on y itself, gives
  // a loop body with 1% fewer instructions: 1.5% faster for float32 and 1%
  // for float64 storage on the 2048x2048 field, same bits.)
  int y = y0;
  for (int i = y0; i < y1 - 1; ++i, ++y) row_step(opaque_row(y), BoolC<true>{});
  row_step(y, BoolC<false>{});  // the last row prefetches nothing
  if (bad) *a.flag = 1;
}

// Workgroups of a launch per XCD: the hardware deals workgroups out to the
// eight XCDs round-robin (workgroup b runs on XCD b % 8).
constexpr int kXcds = 8;

// The rows one XCD walks in a single-grid step, cut into chunks: `rows`
// high (the last one possibly lower) up to the band's last tail_rows rows,
// then short chunks (tail_h high, the last one possibly lower) over those.
// Band x holds rows [x ny / 8, (x + 1) ny / 8).
struct Band {
  int y0, y1;    // the band's rows
  int ys;        // first row of the short chunks
  int nlong;     // chunks of at most `rows` rows in [y0, ys)
  int nchunks;   // long and short
};

__host__ __device__ inline Band band_of(int x, int ny, int rows, int tail_rows, int tail_h) {
  Band b;
  b.y0 = int((long long)x * ny / kXcds);
  b.y1 = int((long long)(x + 1) * ny / kXcds);
  const int t = min(tail_rows, b.y1 - b.y0);
  b.ys = b.y1 - t;
  b.nlong = (b.ys - b.y0 + rows - 1) / rows;
  b.nchunks = b.nlong + (t + tail_h - 1) / tail_h;
  return b;
}

// Grid size of the single-grid step kernel: rounds of kXcds workgroups,
// enough for the band with the most tiles.
template <class P>
int step_grid(const StepArgs<P> &a) {
  int most = 0;
  for (int x = 0; x < kXcds; ++x)
    most = std::max(most, band_of(x, a.ny, a.rows, a.tail_rows, a.tail_h).nchunks);
  return kXcds * ((most * a.nstrips + P::kBlockWaves - 1) / P::kBlockWaves);
}

// One time step of one simulation: one wavefront per tile.  The hardware
// deals workgroups to the XCDs round-robin, so workgroup b runs on XCD
// b % 8 and takes the (b / 8)-th group of tiles of that XCD's band of rows:
// the halo rows a tile shares with the tiles above and below are read
// through the same L2 (measured on 2048x2048, float32 storage: reads past
// L2 fell from 226 to 160 bytes per site at equal speed).  Tiles are
// strip-major (consecutive wavefronts take adjacent strips of the same
// rows, so each row streams contiguously from memory).  Each band is
// dispatched in order, so its last chunks are the ones still running when
// the launch drains; they are short, which shortens the drain.
template <class P, int K, bool GENR, bool HAS_S, bool NS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P::kMinWaves)))
lbm_step_kernel(const StepArgs<P> a) {
  // the wavefront index is the same on every lane: make it a scalar so all
  // row arithmetic and row offsets stay in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const Band b = band_of(int(blockIdx.x % kXcds), a.ny, a.rows, a.tail_rows, a.tail_h);
  const int tile = int(blockIdx.x / kXcds) * P::kBlockWaves + wave;
  const int chunk = tile / a.nstrips;
  if (chunk >= b.nchunks) return;  // whole wavefronts only
  const bool full = chunk < b.nlong;
  const int y0 = full ? b.y0 + chunk * a.rows : b.ys + (chunk - b.nlong) * a.tail_h;
  const int y1 = full ? min(y0 + a.rows, b.ys) : min(y0 + a.tail_h, b.y1);
  step_tile<P, K, GENR, HAS_S, NS>(a, tile - chunk * a.nstrips, y0, y1);
}

// ------------------------------------------------------------ batched step

// A tile of the batched step: which simulation, which strip and row chunk.
struct TileRef {
  int inst, strip, chunk, pad;
};

// Per simulation of a batch: the step arguments for both ping-pong
// parities, the parity at the start of the captured chunk, and how many of
// the chunk's launches it takes part in.
template <class P>
struct BatchInst {
  StepArgs<P> a[2];
  int parity, steps, pad[2];
};

// Constant address space: loads through it with a wavefront-uniform address
// become scalar loads.  The qualifier exists only in the device pass.
#if defined(__HIP_DEVICE_COMPILE__)
#define LBM_CONST __attribute__((address_space(4)))
#else
#define LBM_CONST
#endif

// Launch k of a captured chunk for every simulation of one kernel variant.
// Persistent: gridDim.x * P::kBlockWaves wavefronts walk the tile list with a fixed
// stride; the tile count and the per-simulation descriptors are read from
// device memory (scalar loads), so a captured graph stays valid when the
// batch's membership changes between chunks.  Every wavefront leaves the
// loop after at most ceil(ntiles / stride) tiles.
template <class P, int K, bool GENR, bool HAS_S, bool NS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P::kMinWaves)))
lbm_batch_step_kernel(const BatchInst<P> *insts, const TileRef *tiles, const int *ntiles,
                      int k) {
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int nt = *(const LBM_CONST int *)(ntiles);
  const int stride = int(gridDim.x) * P::kBlockWaves;
  for (int t = int(blockIdx.x) * P::kBlockWaves + wave; t < nt; t += stride) {
    const TileRef tr = ((const LBM_CONST TileRef *)(tiles))[t];
    const LBM_CONST BatchInst<P> *bi =
        (const LBM_CONST BatchInst<P> *)(insts) + tr.inst;
    if (k >= bi->steps) continue;
    const StepArgs<P> a = bi->a[(bi->parity + k) & 1];
    const int y0 = tr.chunk * a.rows;
    step_tile<P, K, GENR, HAS_S, NS>(a, tr.strip, y0, min(y0 + a.rows, a.ny));
  }
}

// ------------------------------------------------------------ site kernels

// Neighbour of site (x, y) at offset (dx, dy) in {-1,0,1}^2: periodic in x;
// periodic in y or, between walls, the wall row itself (mirror ghost).
__device__ __forceinline__ void nbr_xy(int x, int y, int dx, int dy, int nx, int ny,
                                       int walls, int &xx, int &yy) {
  xx = x + dx;
  yy = y + dy;
  xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
  if (walls) {
    yy = yy < 0 ? 0 : (yy >= ny ? ny - 1 : yy);
  } else {
    yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
  }
}

// The 9-point neighbourhood of site (x, y) of a field given by an index
// function idx(y, x).
template <class R, class F>
__device__ __forceinline__ Nine<R> gather9(F get, int x, int y, int nx, int ny, int walls) {
  auto v9 = [&](int dx, int dy) {
    int xx, yy;
    nbr_xy(x, y, dx, dy, nx, ny, walls, xx, yy);
    return R(get(yy, xx));
  };
  Nine<R> v;
  v.mL = v9(-1, -1);
  v.m = v9(0, -1);
  v.mR = v9(1, -1);
  v.cL = v9(-1, 0);
  v.c = v9(0, 0);
  v.cR = v9(1, 0);
  v.nL = v9(-1, 1);
  v.n = v9(0, 1);
  v.nR = v9(1, 1);
  return v;
}

template <class P>
struct SiteArgs {
  const typename P::S *src;
  const typename P::A *src_rest;
  typename P::S *dst;
  typename P::A *dst_rest;
  typename P::A *aux;
  double *scratch;  // kScratch float64 planes
  Scales<P> sc;
  long long plane;
  int nx, ny, walls;
  int ns;  // 1: velocity from the Navier-Stokes LB; 0: prescribed (aux slots 0, 1)
};

// Initial state in float64: post-collision populations := equilibria of
// Eqs. (22), (26), (30) with P = 0 and S of Eq. (16) from the gradient of
// the initial phi; previous level := the initial fields.  Inputs are
// scratch planes 0-3 (phi, psi, ux, uy).  f and g are stored as deviations
// from w_i times the STORED rest value, so storing phi, psi in a narrower
// type leaves the populations themselves exact up to their own rounding.
template <class P>
__global__ void __launch_bounds__(256)
lbm_init_kernel(const SiteArgs<P> a, const Phys<double> p) {
  using A = typename P::A;
  using R = typename P::R;
  const long long n = (long long)a.nx * a.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int nx = a.nx;
  const int x = int(k % nx), y = int(k / nx);
  const long long pl = a.plane;
  const double *phi0 = a.scratch, *psi0 = a.scratch + pl;
  const double *ux0 = a.scratch + 2 * pl, *uy0 = a.scratch + 3 * pl;
  const Nine<double> v = gather9<double>(
      [&](int yy, int xx) { return phi0[(long long)yy * nx + xx]; }, x, y, nx, a.ny, a.walls);
  double gx, gy;
  grad9(v, gx, gy);
  const double phi = phi0[k], psi = psi0[k], ux = ux0[k], uy = uy0[k];
  const double gn = sqrt(gx * gx + gy * gy);
  const double inv = 1.0 / (gn + p.eps_n);
  const double delta = p.c4W * ((p.phiA - phi) * (phi - p.phiB));
  const double Sx = p.Mdrho * (gx - delta * gx * inv);
  const double Sy = p.Mdrho * (gy - delta * gy * inv);
  const double rho = rho_of(p, phi);
  const double jx = rho * ux, jy = rho * uy;
  const double Ax = jx - Sx, Ay = jy - Sy, Au = Ax * ux + Ay * uy;
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double phis = double(A(phi)), psis = double(A(psi));
  // float16 storage: h relative to the rest parts of the STORED (P = 0, rho u)
  R hbase[8] = {};
  if constexpr (P::HDEV) {
    const HRest<R> v = {R(0), R(A(jx)), R(A(jy))};
    h_store_basis(v, hbase);
  }
  for (int i = 0; i < 9; ++i) {
    const double cu = cx[i] * ux + cy[i] * uy;
    st<P>(a.dst, fg_idx(i, 0, y, x, nx), R(w[i] * (phi - phis) + w[i] * phi * 3.0 * cu),
          a.sc.f);
    st<P>(a.dst, fg_idx(i, 1, y, x, nx), R(w[i] * (psi - psis) + w[i] * psi * 3.0 * cu),
          a.sc.g);
    if (i > 0) {
      const double cj = cx[i] * jx + cy[i] * jy;
      const double cA = cx[i] * Ax + cy[i] * Ay;
      st<P>(a.dst, h_idx(i, y, x, nx),
            R(w[i] * (3.0 * cj + 4.5 * cA * cu - 1.5 * Au) - double(hbase[i - 1])), a.sc.h);
    }
  }
  a.dst_rest[rest_idx<P>(0, y, x, nx)] = A(phi);
  a.dst_rest[rest_idx<P>(1, y, x, nx)] = A(psi);
  if (!a.ns) {  // prescribed velocity, held in aux slots 0, 1 for good
    a.aux[aux_idx<P>(0, y, x, nx)] = A(ux);
    a.aux[aux_idx<P>(1, y, x, nx)] = A(uy);
    return;
  }
  if constexpr (P::HDEV) {
    a.dst_rest[rest_idx<P>(2, y, x, nx)] = A(0);
    a.dst_rest[rest_idx<P>(3, y, x, nx)] = A(jx);
    a.dst_rest[rest_idx<P>(4, y, x, nx)] = A(jy);
  } else {
    a.aux[aux_idx<P>(0, y, x, nx)] = A(ux);
    a.aux[aux_idx<P>(1, y, x, nx)] = A(uy);
  }
}

// Read-back, pass 1: phi, psi, sigma of the current level into scratch
// planes 5-7 (arithmetic type R), by the same streaming as the step.
template <class P>
__global__ void __launch_bounds__(256)
lbm_macro_scalars_kernel(const SiteArgs<P> a, const Phys<typename P::R> p) {
  using R = typename P::R;
  const long long n = (long long)a.nx * a.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int nx = a.nx;
  const int x = int(k % nx), y = int(k / nx);
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const long long pl = a.plane;
  const RowN r = row_numbers(y, a.ny, a.walls);
  R d[9], q[9], e[9];
  pull_fg<P>(a.src, r, x, xm, xp, nx, a.sc.fi, a.sc.gi, d, q);
  const auto *rs = a.src_rest;
  const Nine<R> vx = gather9<R>([&](int yy, int xx) { return rs[rest_idx<P>(0, yy, xx, nx)]; },
                                x, y, nx, a.ny, a.walls);
  source_offsets(vx, r.bot, r.top, e);
  const R phi = restream(d, e, vx.c);
  const Nine<R> vy = gather9<R>([&](int yy, int xx) { return rs[rest_idx<P>(1, yy, xx, nx)]; },
                                x, y, nx, a.ny, a.walls);
  source_offsets(vy, r.bot, r.top, e);
  const R psi = restream(q, e, vy.c);
  R *out = reinterpret_cast<R *>(a.scratch + 5 * pl);
  out[k] = phi;
  out[pl + k] = psi;
  out[2 * pl + k] = sigma_of(p, psi);
}

// Read-back, pass 2: u and P by the same closures as the step, float64
// phi, psi, ux, uy, P into scratch planes 0-4.
template <class P, bool HAS_S>
__global__ void __launch_bounds__(256)
lbm_macro_fields_kernel(const SiteArgs<P> a, const Phys<typename P::R> p) {
  using R = typename P::R;
  const long long n = (long long)a.nx * a.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int nx = a.nx;
  const int x = int(k % nx), y = int(k / nx);
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const long long pl = a.plane;
  const R *sc = reinterpret_cast<const R *>(a.scratch + 5 * pl);
  const Nine<R> vphi = gather9<R>([&](int yy, int xx) { return sc[(long long)yy * nx + xx]; },
                                  x, y, nx, a.ny, a.walls);
  const R *ss = sc + 2 * pl;
  const Nine<R> vsig = gather9<R>([&](int yy, int xx) { return ss[(long long)yy * nx + xx]; },
                                  x, y, nx, a.ny, a.walls);
  R gfx, gfy, gsx, gsy;
  grad9(vphi, gfx, gfy);
  grad9(vsig, gsx, gsy);
  const R lphi = lap9(vphi);
  const R php = R(a.src_rest[rest_idx<P>(0, y, x, nx)]);
  const R psp = R(a.src_rest[rest_idx<P>(1, y, x, nx)]);
  if (!a.ns) {  // prescribed velocity: u as given, P = 0
    a.scratch[k] = double(vphi.c);
    a.scratch[pl + k] = double(sc[pl + k]);
    a.scratch[2 * pl + k] = double(a.aux[aux_idx<P>(0, y, x, nx)]);
    a.scratch[3 * pl + k] = double(a.aux[aux_idx<P>(1, y, x, nx)]);
    a.scratch[4 * pl + k] = 0.0;
    return;
  }
  // the previous level's mass flux from the previous phi, as in the step
  R Sxp = R(0), Syp = R(0);
  if constexpr (HAS_S) {
    const auto *rs = a.src_rest;
    const Nine<R> vq = gather9<R>(
        [&](int yy, int xx) { return R(rs[rest_idx<P>(0, yy, xx, nx)]); }, x, y, nx, a.ny,
        a.walls);
    R gqx, gqy;
    grad9(vq, gqx, gqy);
    mass_flux(p, php, gqx, gqy, Sxp, Syp);
  }
  const RowN r = row_numbers(y, a.ny, a.walls);
  R h[8];
  pull_h<P>(a.src, r, x, xm, xp, nx, a.sc.hi, rho_of(p, php), p.uwb, p.uwt, h);
  R uxp, uyp;
  if constexpr (P::HDEV) {
    const auto *rs = a.src_rest;
    auto g = [&](int c) {
      return gather9<R>([&](int yy, int xx) { return rs[rest_idx<P>(c, yy, xx, nx)]; }, x, y,
                        nx, a.ny, a.walls);
    };
    const Nine<R> vP = g(2), vjx = g(3), vjy = g(4);
    R b[8];
    h_arrival_basis(vP, vjx, vjy, r.bot, r.top, b);
    for (int i = 0; i < 8; ++i) h[i] += b[i];
    const R irho = R(1) / rho_of(p, php);
    uxp = vjx.c * irho;
    uyp = vjy.c * irho;
  } else {
    uxp = R(a.aux[aux_idx<P>(0, y, x, nx)]);
    uyp = R(a.aux[aux_idx<P>(1, y, x, nx)]);
  }
  Front<R> s;
  site_front<R, HAS_S>(p, s, vphi.c, sc[pl + k], vsig.c, gfx, gfy, lphi, gsx, gsy, h, php,
                       psp, uxp, uyp, Sxp, Syp);
  a.scratch[k] = double(s.phi);
  a.scratch[pl + k] = double(s.psi);
  a.scratch[2 * pl + k] = double(s.ux);
  a.scratch[3 * pl + k] = double(s.uy);
  a.scratch[4 * pl + k] = double(s.P);
}

// Float64 reductions over scratch planes 0-3 (phi, psi, ux, uy): per-block
// partial sums in a fixed order (wavefront shuffles, then LDS), then one
// block adds the partials in a fixed order.  Deterministic.
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, kWave));
  return v;
}

__global__ void __launch_bounds__(256)
lbm_reduce_kernel(const double *scratch, long long plane, long long n,
                  const Phys<double> p, double *partials) {
  double acc[kReduceVals] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const double phi = scratch[k], psi = scratch[plane + k];
    const double ux = scratch[2 * plane + k], uy = scratch[3 * plane + k];
    const double rho = rho_of(p, phi);
    const double u2 = ux * ux + uy * uy;
    acc[0] += phi;
    acc[1] += psi;
    acc[2] += rho * ux;
    acc[3] += rho * uy;
    acc[4] += 0.5 * rho * u2;
    acc[5] = fmax(acc[5], sqrt(u2));
    if (!isfinite(phi + psi + ux + uy)) acc[6] = 1.0;
  }
  __shared__ double lds[kReduceVals][256 / kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  for (int j = 0; j < 7; ++j) {
    const double v = (j == 5 || j == 6) ? wave_max(acc[j]) : wave_sum(acc[j]);
    if (lane == 0) lds[j][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int j = threadIdx.x;
    double v = lds[j][0];
    for (int q = 1; q < 256 / kWave; ++q)
      v = (j == 5 || j == 6) ? fmax(v, lds[j][q]) : v + lds[j][q];
    partials[blockIdx.x * kReduceVals + j] = v;
  }
}

__global__ void __launch_bounds__(64)
lbm_reduce_final_kernel(const double *partials, int nblocks, double *out) {
  if (threadIdx.x >= 7) return;
  const int j = threadIdx.x;
  double v = partials[j];
  for (int b = 1; b < nblocks; ++b) {
    const double q = partials[b * kReduceVals + j];
    v = (j == 5 || j == 6) ? fmax(v, q) : v + q;
  }
  out[j] = v;
}

// Shape diagnostics of fluid A from the float64 phi of scratch plane 0:
// c = (phi - phiB)/(phiA - phiB).  Pass 1 sums c, c cos/sin of the periodic
// angles of x and y, c y, and |grad phi|; pass 2 sums c dx^2, c dx dy,
// c dy^2 about the centroid (minimum image along periodic directions).
// Per-block partials in a fixed order, as in lbm_reduce_kernel.
constexpr int kShapeVals = 7;
template <int PASS>
__global__ void __launch_bounds__(256)
lbm_shape_kernel(const double *phi, int nx, int ny, int walls, double phiA, double phiB,
                 double cx, double cy, double *partials) {
  double acc[kShapeVals] = {0, 0, 0, 0, 0, 0, 0};
  const long long n = (long long)nx * ny;
  const double inv = 1.0 / (phiA - phiB);
  const double tx = 2.0 * M_PI / nx, ty = 2.0 * M_PI / ny;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int x = int(k % nx), y = int(k / nx);
    const double c = (phi[k] - phiB) * inv;
    if (PASS == 1) {
      const Nine<double> v = gather9<double>(
          [&](int yy, int xx) { return phi[(long long)yy * nx + xx]; }, x, y, nx, ny, walls);
      double gx, gy;
      grad9(v, gx, gy);
      acc[0] += c;
      acc[1] += c * cos(tx * x);
      acc[2] += c * sin(tx * x);
      acc[3] += c * cos(ty * y);
      acc[4] += c * sin(ty * y);
      acc[5] += c * y;
      acc[6] += sqrt(gx * gx + gy * gy);
    } else {
      double dx = x - cx;
      dx -= nx * rint(dx / nx);
      double dy = y - cy;
      if (!walls) dy -= ny * rint(dy / ny);
      acc[0] += c * dx * dx;
      acc[1] += c * dx * dy;
      acc[2] += c * dy * dy;
    }
  }
  __shared__ double lds[kShapeVals][256 / kWave];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x >> 6;
  for (int j = 0; j < kShapeVals; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) lds[j][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < kShapeVals) {
    const int j = threadIdx.x;
    double v = lds[j][0];
    for (int q = 1; q < 256 / kWave; ++q) v += lds[j][q];
    partials[blockIdx.x * kShapeVals + j] = v;
  }
}

// Sums of nvals partial columns over nblocks, in block order.
__global__ void __launch_bounds__(64)
lbm_sum_final_kernel(const double *partials, int nblocks, int nvals, double *out) {
  if (int(threadIdx.x) >= nvals) return;
  const int j = threadIdx.x;
  double v = partials[j];
  for (int b = 1; b < nblocks; ++b) v += partials[b * nvals + j];
  out[j] = v;
}

// ------------------------------------------------------------------ host

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t storage_size(int prec) {
  return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2);
}
size_t field_size(int prec) { return prec == LBM_FP64 ? 8 : 4; }
// fields per site of the rest record (ping-pong) and the aux record
int rest_fields(int prec) { return prec == LBM_FP16DEV ? F16::kRest : F32::kRest; }
int aux_fields(int prec) { return prec == LBM_FP16DEV ? F16::kAux : F32::kAux; }

struct Layout {
  long long plane;  // elements per plane
  size_t pop_bytes, rest_bytes, aux_bytes, scratch_bytes, partial_bytes;
  size_t off_pop[2], off_rest[2], off_aux, off_scratch, off_partial, off_flag, total;
};

Layout make_layout(const lbm_params &p) {
  Layout L;
  const long long n = (long long)p.nx * p.ny;
  L.plane = (long long)align_up((size_t)n, 64);
  L.pop_bytes = align_up((size_t)kPlanes * n * storage_size(p.precision), 256);
  L.rest_bytes = align_up((size_t)rest_fields(p.precision) * n * field_size(p.precision), 256);
  L.aux_bytes = align_up((size_t)aux_fields(p.precision) * n * field_size(p.precision), 256);
  L.scratch_bytes = align_up((size_t)kScratch * L.plane * 8, 256);
  L.partial_bytes = align_up((size_t)(kReduceBlocks + 1) * kReduceVals * 8, 256);
  size_t o = 0;
  for (int c = 0; c < 2; ++c) {
    L.off_pop[c] = o;
    o += L.pop_bytes;
    L.off_rest[c] = o;
    o += L.rest_bytes;
  }
  L.off_aux = o;
  o += L.aux_bytes;
  L.off_scratch = o;
  o += L.scratch_bytes;
  L.off_partial = o;
  o += L.partial_bytes;
  L.off_flag = o;
  o += 256;
  L.total = o;
  return L;
}

std::string g_create_error;

const char *validate(const lbm_params *p) {
  if (!p) return "params is NULL";
  if (p->nx < 3 || p->ny < 3) return "nx and ny must be >= 3";
  if ((long long)p->nx * p->ny > (1LL << 31)) return "grid too large";
  if (p->walls_y != 0 && p->walls_y != 1) return "walls_y must be 0 or 1";
  if (p->eos != LBM_EOS_LINEAR && p->eos != LBM_EOS_LANGMUIR) return "unknown eos";
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32 && p->precision != LBM_FP16DEV)
    return "unknown precision";
  if (p->flow != LBM_FLOW_NS && p->flow != LBM_FLOW_PRESCRIBED) return "unknown flow";
  {
    // the step kernel addresses each population copy through one buffer
    // resource with 32-bit byte offsets, and its halo lanes store at
    // kDropped, which must lie past every resource
    const unsigned long long sites = (unsigned long long)p->nx * p->ny;
    if (kPlanes * sites * storage_size(p->precision) > kDropped)
      return "grid too large: 26 population planes must fit in 4 GiB";
    if (rest_fields(p->precision) * sites * field_size(p->precision) > kDropped)
      return "grid too large: the rest records must fit in 4 GiB";
  }
  if (!(p->phiA > p->phiB)) return "phiA must exceed phiB";
  if (!(p->W > 0)) return "W must be > 0";
  if (!(p->M > 0) || !(p->D > 0)) return "M and D must be > 0 (tau > 1/2)";
  if (!(p->rhoA > 0) || !(p->rhoB > 0)) return "densities must be > 0";
  if (!(p->muA > 0) || !(p->muB > 0)) return "viscosities must be > 0";
  if (!(p->r >= 0)) return "r must be >= 0";
  if (!(p->sigma0 >= 0)) return "sigma0 must be >= 0";
  const double fin[] = {p->u_wall_bot, p->u_wall_top, p->beta, p->gx, p->gy};
  for (double v : fin)
    if (!std::isfinite(v)) return "non-finite parameter";
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (!(p->s_free[a][b] > 0 && p->s_free[a][b] < 2)) return "free rates must lie in (0, 2)";
  for (int a = 0; a < 3; ++a) {
    const double s = p->fp16_scale[a];
    if (s == 0) continue;
    int e;
    if (!(s > 0) || std::frexp(s, &e) != 0.5 || e < -29 || e > 31)  // s = 2^(e-1)
      return "fp16_scale entries must be 0 or powers of two in [2^-30, 2^30]";
  }
  return nullptr;
}

template <class R>
Phys<R> make_phys(const lbm_params &q) {
  Phys<R> p;
  const double dphi = q.phiA - q.phiB;
  const double drho = (q.rhoA - q.rhoB) / dphi;
  p.phiA = R(q.phiA);
  p.phiB = R(q.phiB);
  p.phiAB = R(q.phiA + q.phiB);
  p.c4W = R(4.0 / (q.W * dphi));
  p.cbulk = R(24.0 / (q.W * dphi * dphi * dphi * dphi));
  p.cW = R(1.5 * q.W / (dphi * dphi));
  p.rhoB = R(q.rhoB);
  p.drho = R(drho);
  p.muB = R(q.muB);
  p.dmu = R((q.muA - q.muB) / dphi);
  p.Mdrho = R(q.M * drho);
  p.gx = R(q.gx);
  p.gy = R(q.gy);
  p.sigma0 = R(q.sigma0);
  p.beta = R(q.beta);
  p.r = R(q.r);
  p.rm1 = R(q.r - 1.0);
  p.s1f = R(1.0 / (3.0 * q.M + 0.5));
  p.s2f = R(q.s_free[0][0]);
  p.s3f = R(q.s_free[0][1]);
  p.s4f = R(q.s_free[0][2]);
  p.s1g = R(1.0 / (3.0 * q.D + 0.5));
  p.s2g = R(q.s_free[1][0]);
  p.s3g = R(q.s_free[1][1]);
  p.s4g = R(q.s_free[1][2]);
  p.s3h = R(q.s_free[2][1]);
  p.s4h = R(q.s_free[2][2]);
  p.uwb = R(q.u_wall_bot);
  p.uwt = R(q.u_wall_top);
  p.psi_max = R(1.0 - 1e-9);
  // 1e-4 of the largest gradient of the equilibrium profile: inside drops,
  // where |grad phi| can fall below delta(phi), the sharpening flux must not
  // become anti-diffusive (it would amplify rounding differences)
  p.eps_n = R(1e-4 * dphi / q.W);
  p.eos = q.eos;
  return p;
}

// Default float16 scales: deviations of f and g are at most a few 1e-2 of
// their field, h_i are O(w_i (3P + 3 c.rho u)); the scales put the expected
// magnitudes near 2^4..2^8, well inside float16's normal range.
void fp16_scales(const lbm_params &q, double out[3]) {
  const double dflt[3] = {4096.0, 4096.0, 65536.0};
  for (int a = 0; a < 3; ++a) out[a] = q.fp16_scale[a] > 0 ? q.fp16_scale[a] : dflt[a];
}

template <class P>
Scales<P> make_scales(const lbm_params &q) {
  using R = typename P::R;
  Scales<P> s;
  double v[3] = {1.0, 1.0, 1.0};
  if (P::SCALED) fp16_scales(q, v);
  s.f = R(v[0]);
  s.g = R(v[1]);
  s.h = R(v[2]);
  s.fi = R(1.0 / v[0]);
  s.gi = R(1.0 / v[1]);
  s.hi = R(1.0 / v[2]);
  return s;
}

}  // namespace

struct lbm_handle {
  lbm_params p;
  Layout L;
  hipStream_t stream;
  char *ws;
  int cur;
  int64_t step;
  bool valid;
  int rows;
  int tail_rows, tail_h;  // short chunks at the end of each band (taper_of)
  bool genr, has_s, ns;
  bool resident;  // step stores with the default cache policy (cache_resident)
  int waves_resident;  // step wavefronts the device holds at once (0: unknown)
  std::string kernel;  // the step kernel variant, as a profiler names it
  std::string err;
  double *fixed_scratch;  // this device's copy of the static read-back scratch
};

// Step launches: compiled in both passes of this file (see lbm_f16_part).
namespace {

void *pops(lbm_handle *h, int which) { return h->ws + h->L.off_pop[which]; }
void *rest(lbm_handle *h, int which) { return h->ws + h->L.off_rest[which]; }
void *auxp(lbm_handle *h) { return h->ws + h->L.off_aux; }
double *scratch(lbm_handle *h) { return reinterpret_cast<double *>(h->ws + h->L.off_scratch); }
double *partials(lbm_handle *h) { return reinterpret_cast<double *>(h->ws + h->L.off_partial); }
int *flagp(lbm_handle *h) { return reinterpret_cast<int *>(h->ws + h->L.off_flag); }

// Columns per lane of the step kernel: two for float32 and float16 storage
// when nx is even (each lane's pair of columns then never straddles the
// periodic seam), else one.
int sites_per_lane(const lbm_params &p) {
  return p.precision != LBM_FP64 && p.nx % 2 == 0 ? 2 : 1;
}
// Whether a grid lies where default stores beat non-temporal ones: measured
// for float32 and float64 storage on single grids from 256x128 to 2048^2,
// the default is 6-25% faster (the written populations are read back from
// the Infinity Cache) from 250 k to 1.25 M sites with float32 storage and
// from 125 k to 625 k sites with float64 storage (64-320 MB of step traffic
// at the 256 and 512 bytes per site the step moved when those measurements
// were taken), and equal or slower outside.
bool cache_resident(const lbm_params &p) {
  const double sites = double(p.nx) * double(p.ny);
  if (p.precision == LBM_FP32) return sites >= 250e3 && sites <= 1.25e6;
  if (p.precision == LBM_FP64) return sites >= 125e3 && sites <= 625e3;
  return false;
}

int strips_of(const lbm_params &p) {
  const int cols = sites_per_lane(p) == 2 ? Strip<2>::kCols : Strip<1>::kCols;
  return (p.nx + cols - 1) / cols;
}

// One step launch; with waves_per_cu set, instead the number of this
// variant's wavefronts one compute unit holds at once.
template <class P, int K, bool GENR, bool HAS_S, bool NS>
hipError_t launch_step(lbm_handle *h, int *waves_per_cu) {
  if (waves_per_cu) {
    int blocks = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, lbm_step_kernel<P, K, GENR, HAS_S, NS>, kWave * P::kBlockWaves, 0);
    *waves_per_cu = blocks * P::kBlockWaves;
    return e;
  }
  StepArgs<P> a;
  a.p = make_phys<typename P::R>(h->p);
  a.sc = make_scales<P>(h->p);
  a.src = static_cast<const typename P::S *>(pops(h, h->cur));
  a.src_rest = static_cast<const typename P::A *>(rest(h, h->cur));
  a.dst = static_cast<typename P::S *>(pops(h, h->cur ^ 1));
  a.dst_rest = static_cast<typename P::A *>(rest(h, h->cur ^ 1));
  a.aux = static_cast<typename P::A *>(auxp(h));
  a.flag = flagp(h);
  a.nx = h->p.nx;
  a.ny = h->p.ny;
  a.walls = h->p.walls_y;
  a.nstrips = strips_of(h->p);
  a.rows = h->rows;
  a.tail_rows = h->tail_rows;
  a.tail_h = h->tail_h;
  hipLaunchKernelGGL((lbm_step_kernel<P, K, GENR, HAS_S, NS>), dim3(step_grid<P>(a)),
                     dim3(kWave * P::kBlockWaves), 0, h->stream, a);
  return hipGetLastError();
}

template <class P, int K>
hipError_t launch_step_prec(lbm_handle *h, int *waves_per_cu) {
  if (!h->ns)
    return h->genr ? launch_step<P, K, true, false, false>(h, waves_per_cu)
                   : launch_step<P, K, false, false, false>(h, waves_per_cu);
  if (h->genr)
    return h->has_s ? launch_step<P, K, true, true, true>(h, waves_per_cu)
                    : launch_step<P, K, true, false, true>(h, waves_per_cu);
  return h->has_s ? launch_step<P, K, false, true, true>(h, waves_per_cu)
                  : launch_step<P, K, false, false, true>(h, waves_per_cu);
}

template <class P, int K, bool GENR, bool HAS_S, bool NS>
void launch_batch(int blocks, hipStream_t st, const void *desc, const TileRef *tiles,
                  const int *count, int k) {
  hipLaunchKernelGGL((lbm_batch_step_kernel<P, K, GENR, HAS_S, NS>), dim3(blocks),
                     dim3(kWave * P::kBlockWaves), 0, st,
                     static_cast<const BatchInst<P> *>(desc), tiles, count, k);
}

template <class P, int K>
void launch_batch_prec(int c, int blocks, hipStream_t st, const void *desc,
                       const TileRef *tiles, const int *count, int k) {
  switch (c & 7) {
    case 0: launch_batch<P, K, false, false, true>(blocks, st, desc, tiles, count, k); break;
    case 1: launch_batch<P, K, false, true, true>(blocks, st, desc, tiles, count, k); break;
    case 2: launch_batch<P, K, true, false, true>(blocks, st, desc, tiles, count, k); break;
    case 3: launch_batch<P, K, true, true, true>(blocks, st, desc, tiles, count, k); break;
    case 4: launch_batch<P, K, false, false, false>(blocks, st, desc, tiles, count, k); break;
    default: launch_batch<P, K, true, false, false>(blocks, st, desc, tiles, count, k); break;
  }
}

}  // namespace

// The float16 step kernels are compiled in a second pass of this file
// (LBM_F16_PART) that fuses a multiply and an add only within one source
// expression (-ffp-contract=on, done by the front end and so the same in
// every inlined copy).  Float16 storage rounds stochastically from all 32
// bits of each value, so every copy of the row code must give the same
// bits for the results not to depend on the tile height; the float32 and
// float64 kernels keep the compiler's default fusion (1-2% faster) and are
// tile-height independent with it.
namespace lbm_f16_part {
hipError_t step(lbm_handle *h, int *waves_per_cu);
void batch(int c, int blocks, hipStream_t st, const void *desc, const void *tiles,
           const int *count, int k);
}  // namespace lbm_f16_part

#ifdef LBM_F16_PART
namespace lbm_f16_part {
hipError_t step(lbm_handle *h, int *waves_per_cu) {
  return sites_per_lane(h->p) == 2 ? launch_step_prec<F16, 2>(h, waves_per_cu)
                                   : launch_step_prec<F16, 1>(h, waves_per_cu);
}
void batch(int c, int blocks, hipStream_t st, const void *desc, const void *tiles,
           const int *count, int k) {
  const TileRef *t = static_cast<const TileRef *>(tiles);
  if (c / 8 == int(LBM_FP16DEV))
    launch_batch_prec<F16, 1>(c, blocks, st, desc, t, count, k);
  else
    launch_batch_prec<F16, 2>(c, blocks, st, desc, t, count, k);
}
}  // namespace lbm_f16_part
#else

namespace {

lbm_status fail(lbm_handle *h, lbm_status s, const std::string &msg) {
  if (h)
    h->err = msg;
  else
    g_create_error = msg;
  return s;
}

lbm_status hip_check(lbm_handle *h, hipError_t e, const char *what) {
  if (e == hipSuccess) return LBM_OK;
  return fail(h, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}


template <class P>
SiteArgs<P> site_args(lbm_handle *h) {
  SiteArgs<P> a;
  a.src = static_cast<const typename P::S *>(pops(h, h->cur));
  a.src_rest = static_cast<const typename P::A *>(rest(h, h->cur));
  a.dst = static_cast<typename P::S *>(pops(h, h->cur));
  a.dst_rest = static_cast<typename P::A *>(rest(h, h->cur));
  a.aux = static_cast<typename P::A *>(auxp(h));
  a.scratch = scratch(h);
  a.sc = make_scales<P>(h->p);
  a.plane = h->L.plane;
  a.nx = h->p.nx;
  a.ny = h->p.ny;
  a.walls = h->p.walls_y;
  a.ns = h->ns ? 1 : 0;
  return a;
}


int default_rows(const lbm_params &p, bool in_batch = false) {
  const long long strips = strips_of(p);
  // Many short tiles keep the wavefronts' start-up and drain phases
  // staggered; the two extra halo rows per tile are served mostly from
  // cache.  Measured on 2048x2048: 2 rows for float32 with two columns per
  // lane, 3 with one, 5 for float16 storage with two (1% over 4), 4 for
  // float16 with one and for float64 storage.  In a batch of the serving
  // mix (128^2 to 1024^2) float16 storage with two columns is 2% faster
  // with 4 rows than with 5.
  const long long target = p.precision == LBM_FP32 ? 24576 : 16384;
  const bool two = sites_per_lane(p) == 2;
  const long long lo = p.precision == LBM_FP32 ? (two ? 2 : 3)
                     : p.precision == LBM_FP16DEV && two && !in_batch ? 5 : 4;
  long long rows = strips * p.ny / target;
  if (rows < lo) rows = lo;
  if (rows > 64) rows = 64;
  return int(rows);
}


// One step of h (or, with waves_per_cu set, the occupancy of its kernel).
hipError_t run_step(lbm_handle *h, int *waves_per_cu = nullptr) {
  int *w = waves_per_cu;
  switch (h->p.precision) {
    case LBM_FP64:
      return h->resident ? launch_step_prec<F64C, 1>(h, w) : launch_step_prec<F64, 1>(h, w);
    case LBM_FP32:
      if (sites_per_lane(h->p) == 2)
        return h->resident ? launch_step_prec<F32C, 2>(h, w) : launch_step_prec<F32, 2>(h, w);
      return h->resident ? launch_step_prec<F32C, 1>(h, w) : launch_step_prec<F32, 1>(h, w);
    default: return lbm_f16_part::step(h, w);
  }
}

// Default tile height of a single simulation.  A step costs about one
// wavefront's walk down its tile (3-5 us per row) when every wavefront of
// the launch fits on the device at once, so a grid too small to fill the
// device takes the shortest tiles that still fit in one round (measured:
// 1-row tiles make a 64x64 step 1.5-3x faster than the heights tuned for
// large grids).  Larger grids keep those heights (default_rows).
int single_rows(const lbm_handle *h) {
  const int lo = default_rows(h->p);
  const long long strips = strips_of(h->p);
  if (h->waves_resident <= 0) return lo;
  for (int r = 1; r < lo; ++r)
    if (strips * ((h->p.ny + r - 1) / r) <= h->waves_resident) return r;
  return lo;
}

// Short chunks at the end of each XCD's band of a single-grid step (see
// lbm_step_kernel).  When the last tiles are dispatched, the device holds
// tiles at every stage of their walk and idles for about the length of one
// tile's walk as they finish; 1-row chunks make that walk short.  About
// one round of the XCD's wavefront slots takes short chunks, and at most a
// quarter of the band: more would add the prologue of a tile (rebuilding
// the rows before its first) to more of the grid.  Measured on 2048x2048
// (bitwise the same results): float32 storage 198.6 -> 196.2 us per step
// with 15 rows of 1-row chunks per band, float64 365.8 -> 363.1 us with 3,
// float16 storage unchanged; 512x512 float32, 16 rows of 64 in short
// chunks: 15.8 us, 18.8 without, 17.2 with 48.
void taper_of(lbm_handle *h) {
  h->tail_h = 1;
  h->tail_rows = 0;
  if (h->rows <= h->tail_h || h->waves_resident <= 0) return;
  const long long strips = strips_of(h->p);
  const long long round = h->waves_resident / (kXcds * strips) * h->tail_h;
  h->tail_rows = int(std::min<long long>(round, h->p.ny / kXcds / 4));
}

// Tile plan of a single-grid step: the tile height (single_rows) and the
// short chunks at each band's end (taper_of).  Float16 storage with two
// columns per lane instead gives every wavefront slot of an XCD one tile
// of the band, when such tiles are at most 24 rows high, and walks the few
// rows left over in 1-row chunks after them: that step is short of vector
// issue, and tall tiles rebuild fewer rows before their first.  Measured on
// 2048x2048: 15 tiles of 17 rows per band and 17 one-row tiles, 159.0 us
// per step against 173.6 with 5-row tiles (float32 and float64 storage are
// 15-20% slower with tiles that tall: their halo rows are no longer shared
// through L2); neutral on 1024x1024 (4 rows) and not applied to taller
// bands (2048x4096, 4096x4096: no gain or slower).
void plan_tiles(lbm_handle *h) {
  h->rows = single_rows(h);
  taper_of(h);
  if (h->p.precision != LBM_FP16DEV || sites_per_lane(h->p) != 2 || h->waves_resident <= 0)
    return;
  const long long per_round = h->waves_resident / (kXcds * strips_of(h->p));  // chunks
  const int band = h->p.ny / kXcds;
  if (per_round < 1 || band / per_round < h->rows || band / per_round > 24) return;
  h->rows = int(band / per_round);
  h->tail_rows = int(band - per_round * h->rows);
  h->tail_h = 1;
}

// The template arguments of the step kernel run_step launches for h, in the
// order a profiler prints them: storage, columns per lane, r != 1,
// rho_A != rho_B, Navier-Stokes velocity.
std::string kernel_name_of(const lbm_handle *h) {
  const char *prec = h->p.precision == LBM_FP64   ? (h->resident ? "F64C" : "F64")
                     : h->p.precision == LBM_FP32 ? (h->resident ? "F32C" : "F32")
                                                  : "F16";
  auto b = [](bool v) { return v ? "true" : "false"; };
  return std::string("lbm_step_kernel<") + prec + ", " + std::to_string(sites_per_lane(h->p)) +
         ", " + b(h->genr) + ", " + b(h->has_s) + ", " + b(h->ns) + ">";
}

// Wavefronts of h's step kernel the current device holds at once (0 if the
// runtime cannot tell).
int query_waves_resident(lbm_handle *h) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      run_step(h, &per_cu) != hipSuccess) {
    (void)hipGetLastError();  // leave no error behind for the next call
    return 0;
  }
  return cus * per_cu;
}

template <class P>
hipError_t launch_macros(lbm_handle *h, double *sc, long long plane) {
  SiteArgs<P> a = site_args<P>(h);
  a.scratch = sc;
  a.plane = plane;
  const long long n = (long long)h->p.nx * h->p.ny;
  const int blocks = int((n + 255) / 256);
  const Phys<typename P::R> p = make_phys<typename P::R>(h->p);
  hipLaunchKernelGGL((lbm_macro_scalars_kernel<P>), dim3(blocks), dim3(256), 0, h->stream,
                     a, p);
  if (h->has_s)
    hipLaunchKernelGGL((lbm_macro_fields_kernel<P, true>), dim3(blocks), dim3(256), 0,
                       h->stream, a, p);
  else
    hipLaunchKernelGGL((lbm_macro_fields_kernel<P, false>), dim3(blocks), dim3(256), 0,
                       h->stream, a, p);
  return hipGetLastError();
}

// The macroscopic fields of the current level into kScratch float64 planes
// of `plane` elements at sc (default: the handle's own scratch).
hipError_t run_macros(lbm_handle *h, double *sc, long long plane) {
  switch (h->p.precision) {
    case LBM_FP64: return launch_macros<F64>(h, sc, plane);
    case LBM_FP32: return launch_macros<F32>(h, sc, plane);
    default: return launch_macros<F16>(h, sc, plane);
  }
}
hipError_t run_macros(lbm_handle *h) { return run_macros(h, scratch(h), h->L.plane); }

// Read-back scratch of lbm_moments_async in static device memory, for
// callers that cannot allocate: kScratch float64 planes of at most
// kFixedSites sites, then the reduction partials.  Each device holds its own
// copy for the life of the process (32.1 MiB); host code reaches it only
// through the address hipGetSymbolAddress gives for that device.
constexpr long long kFixedSites = 1LL << 19;
constexpr long long kFixedDoubles = kScratch * kFixedSites + kReduceBlocks * kReduceVals;
static __device__ __align__(256) double fixed_scratch[kFixedDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
double *g_fixed_ptr[kMaxDevices];  // per device, resolved once

// This device's address of fixed_scratch (nullptr if it cannot be had),
// resolved once per device with that device current.
double *fixed_scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_fixed_mu);
  if (!g_fixed_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(fixed_scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_fixed_ptr[dev] = static_cast<double *>(ptr);
  }
  return g_fixed_ptr[dev];
}

template <class P>
hipError_t launch_init(lbm_handle *h) {
  SiteArgs<P> a = site_args<P>(h);
  const long long n = (long long)h->p.nx * h->p.ny;
  const Phys<double> p = make_phys<double>(h->p);
  hipLaunchKernelGGL((lbm_init_kernel<P>), dim3(int((n + 255) / 256)), dim3(256), 0,
                     h->stream, a, p);
  return hipGetLastError();
}

hipError_t run_init(lbm_handle *h) {
  switch (h->p.precision) {
    case LBM_FP64: return launch_init<F64>(h);
    case LBM_FP32: return launch_init<F32>(h);
    default: return launch_init<F16>(h);
  }
}

// Reads the sticky device flag (synchronising); marks the state invalid.
lbm_status check_flag(lbm_handle *h) {
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, flagp(h), sizeof(int), hipMemcpyDeviceToHost,
                                h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "reading the non-finite flag");
  if (flag) {
    h->valid = false;
    return fail(h, LBM_ENONFINITE, "the device produced a non-finite value");
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params *params) {
  if (validate(params)) return 0;
  return make_layout(*params).total;
}

lbm_status lbm_create(const lbm_params *params, void *dev_ws, size_t ws_bytes,
                      void *hip_stream, lbm_handle **out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char *m = validate(params)) return fail(nullptr, LBM_EINVAL, m);
  const Layout L = make_layout(*params);
  if (!dev_ws) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev_ws) % 256)
    return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < L.total) return fail(nullptr, LBM_ENOMEM, "workspace too small");
  lbm_handle *h = new (std::nothrow) lbm_handle();
  if (!h) return fail(nullptr, LBM_ENOMEM, "out of host memory");
  h->p = *params;
  h->L = L;
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->ws = static_cast<char *>(dev_ws);
  h->cur = 0;
  h->step = 0;
  h->valid = false;
  h->rows = default_rows(*params);
  h->genr = params->r != 1.0;
  h->ns = params->flow == LBM_FLOW_NS;
  h->has_s = h->ns && params->rhoA != params->rhoB;
  h->resident = cache_resident(*params);
  h->waves_resident = query_waves_resident(h);
  plan_tiles(h);
  h->kernel = kernel_name_of(h);
  int dev = -1;
  h->fixed_scratch = hipStreamGetDevice(h->stream, &dev) == hipSuccess ? fixed_scratch_of(dev)
                                                                      : nullptr;
  (void)hipGetLastError();
  *out = h;
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_handle *h, const double *phi, const double *psi,
                           const double *ux, const double *uy) {
  if (!h) return LBM_EINVAL;
  if (!phi || !psi || !ux || !uy) return fail(h, LBM_EINVAL, "NULL field");
  const long long n = (long long)h->p.nx * h->p.ny;
  for (long long k = 0; k < n; ++k) {
    if (!std::isfinite(phi[k]) || !std::isfinite(psi[k]) || !std::isfinite(ux[k]) ||
        !std::isfinite(uy[k]))
      return fail(h, LBM_EINVAL, "non-finite initial value");
    if (h->p.eos == LBM_EOS_LANGMUIR && psi[k] >= 1.0)
      return fail(h, LBM_EINVAL, "Langmuir EOS needs psi < 1");
  }
  double *sc = scratch(h);
  const long long pl = h->L.plane;
  const double *src[4] = {phi, psi, ux, uy};
  for (int j = 0; j < 4; ++j) {
    hipError_t e = hipMemcpyAsync(sc + j * pl, src[j], n * sizeof(double),
                                  hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return hip_check(h, e, "copying initial fields");
  }
  // from here on the stored state is being replaced: a failure leaves no
  // valid state (LBM_ESTATE until a later init or set_state succeeds)
  h->valid = false;
  h->cur = 0;
  hipError_t e = run_init(h);
  if (e == hipSuccess) e = hipMemsetAsync(flagp(h), 0, sizeof(int), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "initialising");
  h->step = 0;
  h->valid = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_handle *h, int64_t nsteps) {
  if (!h) return LBM_EINVAL;
  if (nsteps < 0) return fail(h, LBM_EINVAL, "nsteps < 0");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  for (int64_t t = 0; t < nsteps; ++t) {
    hipError_t e = run_step(h);
    if (e != hipSuccess) {
      // the launches already enqueued still run: the state is no longer the
      // one before the call, nor a known number of steps past it
      if (t > 0) h->valid = false;
      return hip_check(h, e, "launching the step kernel");
    }
    h->cur ^= 1;
    h->step += 1;
  }
  return LBM_OK;
}

lbm_status lbm_read_fields(lbm_handle *h, double *phi, double *psi, double *ux,
                           double *uy, double *P) {
  if (!h) return LBM_EINVAL;
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  lbm_status st = check_flag(h);
  if (st != LBM_OK) return st;
  hipError_t e = run_macros(h);
  if (e != hipSuccess) return hip_check(h, e, "launching read-back kernels");
  const long long n = (long long)h->p.nx * h->p.ny;
  double *dst[5] = {phi, psi, ux, uy, P};
  for (int j = 0; j < 5; ++j) {
    if (!dst[j]) continue;
    e = hipMemcpyAsync(dst[j], scratch(h) + j * h->L.plane, n * sizeof(double),
                       hipMemcpyDeviceToHost, h->stream);
    if (e != hipSuccess) return hip_check(h, e, "copying fields");
  }
  e = hipStreamSynchronize(h->stream);
  return hip_check(h, e, "reading fields");
}

lbm_status lbm_moments(lbm_handle *h, lbm_moments_t *out) {
  if (!h) return LBM_EINVAL;
  if (!out) return fail(h, LBM_EINVAL, "out is NULL");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  lbm_status st = check_flag(h);
  if (st != LBM_OK) return st;
  hipError_t e = run_macros(h);
  if (e != hipSuccess) return hip_check(h, e, "launching read-back kernels");
  const Phys<double> p = make_phys<double>(h->p);
  double *part = partials(h);
  const long long n = (long long)h->p.nx * h->p.ny;
  hipLaunchKernelGGL(lbm_reduce_kernel, dim3(kReduceBlocks), dim3(256), 0, h->stream,
                     (const double *)scratch(h), h->L.plane, n, p, part);
  hipLaunchKernelGGL(lbm_reduce_final_kernel, dim3(1), dim3(64), 0, h->stream,
                     (const double *)part, kReduceBlocks, part + kReduceBlocks * kReduceVals);
  e = hipGetLastError();
  double v[kReduceVals];
  if (e == hipSuccess)
    e = hipMemcpyAsync(v, part + kReduceBlocks * kReduceVals, sizeof v,
                       hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "reducing");
  out->step = h->step;
  out->sum_phi = v[0];
  out->sum_psi = v[1];
  out->mom_x = v[2];
  out->mom_y = v[3];
  out->kinetic = v[4];
  out->max_u = v[5];
  out->nonfinite = v[6] != 0.0;
  out->pad = 0;
  if (out->nonfinite) {
    h->valid = false;
    return fail(h, LBM_ENONFINITE, "non-finite macroscopic field");
  }
  return LBM_OK;
}

lbm_status lbm_moments_async(lbm_handle *h, double *dev_out) {
  if (!h) return LBM_EINVAL;
  if (!dev_out) return fail(h, LBM_EINVAL, "dev_out is NULL");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  const long long n = (long long)h->p.nx * h->p.ny;
  if (n > kFixedSites)
    return fail(h, LBM_EINVAL, "grid has more than 524288 sites, the capacity of the static "
                               "read-back scratch of lbm_moments_async (use lbm_moments)");
  double *base = h->fixed_scratch;
  if (!base) return fail(h, LBM_EDEVICE, "no address of the static read-back scratch");
  const long long plane = (long long)align_up((size_t)n, 64);
  hipError_t e = run_macros(h, base, plane);
  if (e != hipSuccess) return hip_check(h, e, "launching read-back kernels");
  double *part = base + kScratch * kFixedSites;
  const Phys<double> p = make_phys<double>(h->p);
  hipLaunchKernelGGL(lbm_reduce_kernel, dim3(kReduceBlocks), dim3(256), 0, h->stream,
                     (const double *)base, plane, n, p, part);
  hipLaunchKernelGGL(lbm_reduce_final_kernel, dim3(1), dim3(64), 0, h->stream,
                     (const double *)part, kReduceBlocks, dev_out);
  return hip_check(h, hipGetLastError(), "launching the reductions");
}

lbm_status lbm_shape(lbm_handle *h, lbm_shape_t *out) {
  if (!h) return LBM_EINVAL;
  if (!out) return fail(h, LBM_EINVAL, "out is NULL");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  lbm_status st = check_flag(h);
  if (st != LBM_OK) return st;
  hipError_t e = run_macros(h);
  if (e != hipSuccess) return hip_check(h, e, "launching read-back kernels");
  const lbm_params &p = h->p;
  const double *phi = scratch(h);
  double *part = partials(h);
  double *res = part + kReduceBlocks * kShapeVals;
  auto pass = [&](int which, double cx, double cy, double *v) -> hipError_t {
    if (which == 1)
      hipLaunchKernelGGL(lbm_shape_kernel<1>, dim3(kReduceBlocks), dim3(256), 0, h->stream,
                         phi, p.nx, p.ny, p.walls_y, p.phiA, p.phiB, cx, cy, part);
    else
      hipLaunchKernelGGL(lbm_shape_kernel<2>, dim3(kReduceBlocks), dim3(256), 0, h->stream,
                         phi, p.nx, p.ny, p.walls_y, p.phiA, p.phiB, cx, cy, part);
    hipLaunchKernelGGL(lbm_sum_final_kernel, dim3(1), dim3(64), 0, h->stream,
                       (const double *)part, kReduceBlocks, kShapeVals, res);
    hipError_t e2 = hipGetLastError();
    if (e2 == hipSuccess)
      e2 = hipMemcpyAsync(v, res, sizeof(double) * kShapeVals, hipMemcpyDeviceToHost, h->stream);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(h->stream);
    return e2;
  };
  double s1[kShapeVals], s2[kShapeVals];
  e = pass(1, 0.0, 0.0, s1);
  if (e != hipSuccess) return hip_check(h, e, "shape pass 1");
  const double area = s1[0];
  if (!(area > 0.0)) return fail(h, LBM_EINVAL, "no fluid A in the domain");
  auto circ = [](double c, double s, int n) {
    double a = std::atan2(s, c) * n / (2.0 * M_PI);
    a = std::fmod(a, double(n));
    return a < 0 ? a + n : a;
  };
  const double cx = circ(s1[1], s1[2], p.nx);
  const double cy = p.walls_y ? s1[5] / area : circ(s1[3], s1[4], p.ny);
  e = pass(2, cx, cy, s2);
  if (e != hipSuccess) return hip_check(h, e, "shape pass 2");
  const double ixx = s2[0] / area, ixy = s2[1] / area, iyy = s2[2] / area;
  const double tr = ixx + iyy, det = ixx * iyy - ixy * ixy;
  const double disc = std::sqrt(std::max(tr * tr / 4 - det, 0.0));
  const double L = 2 * std::sqrt(tr / 2 + disc), B = 2 * std::sqrt(std::max(tr / 2 - disc, 0.0));
  out->area = area;
  out->cx = cx;
  out->cy = cy;
  out->Ixx = ixx;
  out->Ixy = ixy;
  out->Iyy = iyy;
  out->length = s1[6] / (p.phiA - p.phiB);
  out->taylor_D = (L + B) > 0 ? (L - B) / (L + B) : 0.0;
  out->angle = 0.5 * std::atan2(2 * ixy, ixx - iyy);
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_handle *h) {
  if (!h) return 0;
  return sizeof(int64_t) + h->L.pop_bytes + h->L.rest_bytes + h->L.aux_bytes;
}

lbm_status lbm_get_state(lbm_handle *h, void *host_buf, size_t bytes) {
  if (!h) return LBM_EINVAL;
  if (!host_buf || bytes != lbm_state_bytes(h)) return fail(h, LBM_EINVAL, "bad buffer");
  if (!h->valid) return fail(h, LBM_ESTATE, "no valid state");
  lbm_status st = check_flag(h);
  if (st != LBM_OK) return st;
  char *b = static_cast<char *>(host_buf);
  std::memcpy(b, &h->step, sizeof(int64_t));
  b += sizeof(int64_t);
  const void *parts[3] = {pops(h, h->cur), rest(h, h->cur), auxp(h)};
  const size_t sizes[3] = {h->L.pop_bytes, h->L.rest_bytes, h->L.aux_bytes};
  hipError_t e = hipSuccess;
  for (int j = 0; j < 3 && e == hipSuccess; ++j) {
    e = hipMemcpyAsync(b, parts[j], sizes[j], hipMemcpyDeviceToHost, h->stream);
    b += sizes[j];
  }
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  return hip_check(h, e, "saving state");
}

lbm_status lbm_set_state(lbm_handle *h, const void *host_buf, size_t bytes) {
  if (!h) return LBM_EINVAL;
  if (!host_buf || bytes != lbm_state_bytes(h)) return fail(h, LBM_EINVAL, "bad buffer");
  const char *b = static_cast<const char *>(host_buf);
  int64_t step;
  std::memcpy(&step, b, sizeof(int64_t));
  b += sizeof(int64_t);
  // the stored state is overwritten from here on: a failure leaves no valid
  // state (LBM_ESTATE until a later init or set_state succeeds)
  h->valid = false;
  h->cur = 0;
  void *parts[3] = {pops(h, 0), rest(h, 0), auxp(h)};
  const size_t sizes[3] = {h->L.pop_bytes, h->L.rest_bytes, h->L.aux_bytes};
  hipError_t e = hipSuccess;
  for (int j = 0; j < 3 && e == hipSuccess; ++j) {
    e = hipMemcpyAsync(parts[j], b, sizes[j], hipMemcpyHostToDevice, h->stream);
    b += sizes[j];
  }
  if (e == hipSuccess) e = hipMemsetAsync(flagp(h), 0, sizeof(int), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "restoring state");
  h->step = step;
  h->valid = true;
  return LBM_OK;
}

void lbm_destroy(lbm_handle *h) {
  if (!h) return;
  // work enqueued by lbm_step may still be writing the caller's workspace;
  // finish it before the caller can release or reuse that memory
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

const char *lbm_last_error(const lbm_handle *h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

lbm_status lbm_set_tile_rows(lbm_handle *h, int32_t rows) {
  if (!h) return LBM_EINVAL;
  if (rows < 0 || rows > 4096) return fail(h, LBM_EINVAL, "rows out of range");
  if (rows == 0) {
    plan_tiles(h);
  } else {
    h->rows = rows;
    taper_of(h);
  }
  return LBM_OK;
}

lbm_status lbm_get_tile_plan(const lbm_handle *h, int32_t *plan) {
  if (!h || !plan) return LBM_EINVAL;
  plan[0] = h->rows;
  plan[1] = h->tail_rows;
  plan[2] = h->tail_h;
  return LBM_OK;
}

const char *lbm_step_kernel_name(const lbm_handle *h) {
  return h ? h->kernel.c_str() : "lbm_step_kernel";
}

}  // extern "C"

// ------------------------------------------------------------ batch runtime

namespace {

// Kernel variants: storage precision x prescribed velocity x (r != 1) x
// (rho_A != rho_B); float32 and float16 storage with two columns per lane
// are a fourth and a fifth group after the three precisions.
constexpr int kClasses = 40;
int class_of(const lbm_handle *h) {
  int group = int(h->p.precision);
  if (sites_per_lane(h->p) == 2) group = h->p.precision == LBM_FP32 ? 3 : 4;
  return group * 8 + (h->ns ? 0 : 4) + (h->genr ? 2 : 0) + (h->has_s ? 1 : 0);
}

template <class P>
StepArgs<P> step_args(const lbm_handle *h, int cur) {
  lbm_handle *hh = const_cast<lbm_handle *>(h);
  StepArgs<P> a;
  a.p = make_phys<typename P::R>(h->p);
  a.sc = make_scales<P>(h->p);
  a.src = static_cast<const typename P::S *>(pops(hh, cur));
  a.src_rest = static_cast<const typename P::A *>(rest(hh, cur));
  a.dst = static_cast<typename P::S *>(pops(hh, cur ^ 1));
  a.dst_rest = static_cast<typename P::A *>(rest(hh, cur ^ 1));
  a.aux = static_cast<typename P::A *>(auxp(hh));
  a.flag = flagp(hh);
  a.nx = h->p.nx;
  a.ny = h->p.ny;
  a.walls = h->p.walls_y;
  a.nstrips = strips_of(h->p);
  a.rows = h->rows;
  a.tail_rows = 0;  // batched tiles come from the tile list
  a.tail_h = 1;
  return a;
}

size_t desc_size(int prec) {
  switch (prec) {
    case LBM_FP64: return sizeof(BatchInst<F64>);
    case LBM_FP32: return sizeof(BatchInst<F32>);
    default: return sizeof(BatchInst<F16>);
  }
}

template <class P>
void fill_desc(void *dst, const lbm_handle *h, int steps) {
  BatchInst<P> d;
  std::memset(&d, 0, sizeof d);
  d.a[0] = step_args<P>(h, 0);
  d.a[1] = step_args<P>(h, 1);
  d.parity = h->cur;
  d.steps = steps;
  std::memcpy(dst, &d, sizeof d);
}


// Storage precision of a kernel variant class (its descriptor array).
int class_precision(int c) {
  const int g = c / 8;
  return g == 3 ? int(LBM_FP32) : (g == 4 ? int(LBM_FP16DEV) : g);
}

void launch_batch_class(int c, int blocks, hipStream_t st, const void *desc,
                        const TileRef *tiles, const int *count, int k) {
  switch (c / 8) {
    case LBM_FP64: launch_batch_prec<F64, 1>(c, blocks, st, desc, tiles, count, k); break;
    case LBM_FP32: launch_batch_prec<F32, 1>(c, blocks, st, desc, tiles, count, k); break;
    case 3: launch_batch_prec<F32, 2>(c, blocks, st, desc, tiles, count, k); break;
    default: lbm_f16_part::batch(c, blocks, st, desc, tiles, count, k); break;
  }
}

}  // namespace

struct lbm_batch {
  hipStream_t stream = nullptr;   // the caller's stream: all work goes here
  hipStream_t capture = nullptr;  // library stream used only to record graphs
  hipStream_t admit = nullptr;    // library stream for joiners' copies and init
  char *ws = nullptr;
  size_t ws_bytes = 0;
  int max_inst = 0;
  lbm_host::Arena arena;
  struct Inst {
    lbm_handle *h = nullptr;  // nullptr: free id
    size_t off = 0, bytes = 0;
    int64_t remaining = 0;
    int up_steps = -1, up_parity = -1;  // what the device descriptor holds
  };
  std::vector<Inst> inst;
  // device metadata (from the workspace) and pinned host staging
  size_t meta_off = 0, meta_bytes = 0;
  char *d_desc[3] = {nullptr, nullptr, nullptr};
  int *d_count = nullptr;
  TileRef *d_tiles = nullptr;
  size_t tiles_off = 0, tiles_cap = 0;
  char *h_desc[3] = {nullptr, nullptr, nullptr};
  int *h_count = nullptr;
  TileRef *h_tiles = nullptr;
  size_t h_tiles_cap = 0;
  int class_off[kClasses] = {}, class_n[kClasses] = {};
  bool tiles_dirty = true;
  lbm_schedule sched = {0, 0, 32, 0};
  int cus = 256;
  std::map<std::string, hipGraphExec_t> graphs;
  std::string err;
};

namespace {

lbm_status bfail(const lbm_batch *b, lbm_status s, const std::string &msg) {
  if (b)
    const_cast<lbm_batch *>(b)->err = msg;
  else
    g_create_error = msg;
  return s;
}

lbm_status bhip(lbm_batch *b, hipError_t e, const char *what) {
  if (e == hipSuccess) return LBM_OK;
  return bfail(b, LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void clear_graphs(lbm_batch *b) {
  for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  b->graphs.clear();
}

size_t meta_bytes_for(int max_inst) {
  size_t m = 0;
  for (int p = 0; p < 3; ++p) m += align_up(desc_size(p) * size_t(max_inst), 256);
  return m + align_up(sizeof(int) * kClasses, 256);
}

// Rebuild the tile lists (after a change of membership or schedule):
// simulations grouped by kernel variant, each strip-major.
lbm_status rebuild_tiles(lbm_batch *b) {
  size_t total = 0;
  for (auto &in : b->inst) {
    if (!in.h) continue;
    lbm_handle *h = in.h;
    h->rows = b->sched.rows > 0 ? b->sched.rows : default_rows(h->p, true);
    const size_t strips = strips_of(h->p);
    total += strips * size_t((h->p.ny + h->rows - 1) / h->rows);
  }
  hipError_t e = hipStreamSynchronize(b->stream);  // staging and tiles idle
  if (e != hipSuccess) return bhip(b, e, "synchronising");
  if (total > b->tiles_cap) {  // grow the device tile list
    const size_t cap = std::max(total, 2 * b->tiles_cap);
    if (b->d_tiles) b->arena.release(b->tiles_off, b->tiles_cap * sizeof(TileRef));
    b->d_tiles = nullptr;
    b->tiles_cap = 0;
    size_t off;
    if (!b->arena.alloc_top(cap * sizeof(TileRef), &off))
      return bfail(b, LBM_ENOMEM, "workspace too small for the tile list");
    b->tiles_off = off;
    b->tiles_cap = cap;
    b->d_tiles = reinterpret_cast<TileRef *>(b->ws + off);
    clear_graphs(b);
  }
  if (total > b->h_tiles_cap) {
    const size_t cap = std::max(total, 2 * b->h_tiles_cap);
    if (b->h_tiles) (void)hipHostFree(b->h_tiles);
    b->h_tiles = nullptr;
    b->h_tiles_cap = 0;
    e = hipHostMalloc(reinterpret_cast<void **>(&b->h_tiles), cap * sizeof(TileRef));
    if (e != hipSuccess) return bhip(b, e, "allocating pinned staging");
    b->h_tiles_cap = cap;
  }
  size_t n = 0;
  for (int c = 0; c < kClasses; ++c) {
    b->class_off[c] = int(n);
    for (int id = 0; id < b->max_inst; ++id) {
      const lbm_handle *h = b->inst[id].h;
      if (!h || class_of(h) != c) continue;
      const int strips = strips_of(h->p);
      const int chunks = (h->p.ny + h->rows - 1) / h->rows;
      for (int ch = 0; ch < chunks; ++ch)
        for (int st = 0; st < strips; ++st) b->h_tiles[n++] = TileRef{id, st, ch, 0};
    }
    b->class_n[c] = int(n) - b->class_off[c];
    b->h_count[c] = b->class_n[c];
  }
  if (n) {
    e = hipMemcpyAsync(b->d_tiles, b->h_tiles, n * sizeof(TileRef), hipMemcpyHostToDevice,
                       b->stream);
    if (e != hipSuccess) return bhip(b, e, "uploading tiles");
  }
  e = hipMemcpyAsync(b->d_count, b->h_count, sizeof(int) * kClasses, hipMemcpyHostToDevice,
                     b->stream);
  if (e != hipSuccess) return bhip(b, e, "uploading tile counts");
  for (auto &in : b->inst) in.up_steps = -1;  // rows may have changed
  b->tiles_dirty = false;
  return LBM_OK;
}

// Upload the descriptors of simulations whose (parity, steps this chunk)
// changed.  Synchronises only when something must be written.
lbm_status update_descs(lbm_batch *b, int K) {
  bool need = false;
  for (auto &in : b->inst)
    if (in.h && (in.up_steps != int(std::min<int64_t>(K, in.remaining)) ||
                 in.up_parity != in.h->cur))
      need = true;
  if (!need) return LBM_OK;
  hipError_t e = hipStreamSynchronize(b->stream);  // staging idle
  if (e != hipSuccess) return bhip(b, e, "synchronising");
  for (int id = 0; id < b->max_inst; ++id) {
    auto &in = b->inst[id];
    if (!in.h) continue;
    const int steps = int(std::min<int64_t>(K, in.remaining));
    if (in.up_steps == steps && in.up_parity == in.h->cur) continue;
    const int p = in.h->p.precision;
    char *hd = b->h_desc[p] + size_t(id) * desc_size(p);
    switch (p) {
      case LBM_FP64: fill_desc<F64>(hd, in.h, steps); break;
      case LBM_FP32: fill_desc<F32>(hd, in.h, steps); break;
      default: fill_desc<F16>(hd, in.h, steps); break;
    }
    e = hipMemcpyAsync(b->d_desc[p] + size_t(id) * desc_size(p), hd, desc_size(p),
                       hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return bhip(b, e, "uploading descriptors");
    in.up_steps = steps;
    in.up_parity = in.h->cur;
  }
  return LBM_OK;
}

int class_blocks(const lbm_batch *b, int c) {
  const int waves = b->sched.grid_waves > 0 ? b->sched.grid_waves : b->class_n[c];
  const int prec = class_precision(c);
  const int wpb = prec == LBM_FP16DEV ? F16::kBlockWaves
                : prec == LBM_FP64    ? F64::kBlockWaves
                                      : F32::kBlockWaves;
  return std::max(1, (waves + wpb - 1) / wpb);
}

// The graph of K launches of every variant present, captured once per
// (K, variants, grid shape, tile storage).
lbm_status get_graph(lbm_batch *b, int K, hipGraphExec_t *out) {
  std::string key = std::to_string(K) + ":" + std::to_string(b->sched.grid_waves) + ":" +
                    std::to_string(reinterpret_cast<uintptr_t>(b->d_tiles));
  for (int c = 0; c < kClasses; ++c) {
    key += ":";
    if (b->class_n[c]) key += std::to_string(b->class_off[c]) + "/" +
                              std::to_string(class_blocks(b, c));
  }
  auto it = b->graphs.find(key);
  if (it != b->graphs.end()) {
    *out = it->second;
    return LBM_OK;
  }
  if (b->graphs.size() >= 32) clear_graphs(b);
  hipError_t e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bhip(b, e, "beginning graph capture");
  for (int k = 0; k < K; ++k)
    for (int c = 0; c < kClasses; ++c) {
      if (!b->class_n[c]) continue;
      launch_batch_class(c, class_blocks(b, c), b->capture, b->d_desc[class_precision(c)],
                         b->d_tiles + b->class_off[c], b->d_count + c, k);
    }
  hipGraph_t g = nullptr;
  hipError_t e2 = hipGetLastError();
  e = hipStreamEndCapture(b->capture, &g);
  if (e2 != hipSuccess) e = e2;
  hipGraphExec_t x = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) return bhip(b, e, "capturing the batch graph");
  b->graphs[key] = x;
  *out = x;
  return LBM_OK;
}

bool schedule_ok(const lbm_schedule *s) {
  return s && s->rows >= 0 && s->rows <= 4096 && s->grid_waves >= 0 &&
         s->grid_waves <= (1 << 22) && s->chunk >= 1 && s->chunk <= 1024 && s->reserved == 0;
}

}  // namespace

extern "C" {

size_t lbm_batch_instance_bytes(const lbm_params *params) {
  return lbm_workspace_bytes(params);
}

size_t lbm_batch_overhead_bytes(int32_t max_instances) {
  if (max_instances < 1 || max_instances > 65536) return 0;
  return meta_bytes_for(max_instances);
}

lbm_status lbm_batch_create(int32_t max_instances, void *dev_ws, size_t ws_bytes,
                            void *hip_stream, lbm_batch **out) {
  if (!out) return bfail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_instances < 1 || max_instances > 65536)
    return bfail(nullptr, LBM_EINVAL, "max_instances must be in 1..65536");
  if (!dev_ws) return bfail(nullptr, LBM_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(dev_ws) % 256)
    return bfail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
  const size_t meta = meta_bytes_for(max_instances);
  if (ws_bytes < meta) return bfail(nullptr, LBM_ENOMEM, "workspace smaller than metadata");
  lbm_batch *b = new (std::nothrow) lbm_batch();
  if (!b) return bfail(nullptr, LBM_ENOMEM, "out of host memory");
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->ws = static_cast<char *>(dev_ws);
  b->ws_bytes = ws_bytes;
  b->max_inst = max_instances;
  b->inst.resize(max_instances);
  b->arena.reset(ws_bytes);
  size_t off = 0;
  b->arena.alloc(meta, &off);  // first block: offset 0
  b->meta_off = off;
  b->meta_bytes = meta;
  size_t o = off;
  for (int p = 0; p < 3; ++p) {
    b->d_desc[p] = b->ws + o;
    o += align_up(desc_size(p) * size_t(max_instances), 256);
  }
  b->d_count = reinterpret_cast<int *>(b->ws + o);
  hipError_t e = hipSuccess;
  for (int p = 0; p < 3 && e == hipSuccess; ++p)
    e = hipHostMalloc(reinterpret_cast<void **>(&b->h_desc[p]),
                      desc_size(p) * size_t(max_instances));
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&b->h_count), sizeof(int) * kClasses);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->admit, hipStreamNonBlocking);
  int dev = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    const std::string m = std::string("creating the batch: ") + hipGetErrorString(e);
    lbm_batch_destroy(b);
    return bfail(nullptr, LBM_EDEVICE, m);
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_submit(lbm_batch *b, const lbm_params *params, const double *phi,
                            const double *psi, const double *ux, const double *uy,
                            int64_t nsteps, int32_t *id) {
  if (!b) return LBM_EINVAL;
  if (!id) return bfail(b, LBM_EINVAL, "id is NULL");
  if (nsteps < 0) return bfail(b, LBM_EINVAL, "nsteps < 0");
  if (const char *m = validate(params)) return bfail(b, LBM_EINVAL, m);
  int slot = -1;
  for (int i = 0; i < b->max_inst; ++i)
    if (!b->inst[i].h) {
      slot = i;
      break;
    }
  if (slot < 0) return bfail(b, LBM_ENOMEM, "no free simulation id");
  const size_t bytes = lbm_workspace_bytes(params);
  size_t off;
  if (!b->arena.alloc(bytes, &off))
    return bfail(b, LBM_ENOMEM, "not enough contiguous free workspace");
  // The new simulation's fields are copied in and initialised on the
  // batch's admission stream, so the simulations already stepping on the
  // caller's stream keep running meanwhile.  Its block of the workspace is
  // free of device work: a retire releases a block only after the stream
  // has finished every launch that used it.  It joins the launches of the
  // next lbm_batch_step, which are enqueued after this call has waited for
  // the initialisation to complete.
  lbm_handle *h = nullptr;
  lbm_status st = lbm_create(params, b->ws + off, bytes, b->admit, &h);
  if (st == LBM_OK) {
    st = lbm_init_fields(h, phi, psi, ux, uy);
    if (st != LBM_OK) {
      bfail(b, st, h->err);
      lbm_destroy(h);
      h = nullptr;
    }
  } else {
    bfail(b, st, g_create_error);
  }
  if (st != LBM_OK) {
    b->arena.release(off, bytes);
    return st;
  }
  h->stream = b->stream;  // reads and steps from now on go to the caller's stream
  auto &in = b->inst[slot];
  in.h = h;
  in.off = off;
  in.bytes = bytes;
  in.remaining = nsteps;
  in.up_steps = in.up_parity = -1;
  b->tiles_dirty = true;
  *id = slot;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps) {
  if (!b) return LBM_EINVAL;
  if (nsteps < 0) return bfail(b, LBM_EINVAL, "nsteps < 0");
  while (nsteps > 0) {
    int64_t most = 0;
    for (auto &in : b->inst)
      if (in.h) most = std::max(most, in.remaining);
    if (most == 0) break;  // nothing left to run
    if (b->tiles_dirty) {
      lbm_status st = rebuild_tiles(b);
      if (st != LBM_OK) return st;
    }
    const int K = int(std::min<int64_t>({nsteps, int64_t(b->sched.chunk), most}));
    lbm_status st = update_descs(b, K);
    if (st != LBM_OK) return st;
    hipGraphExec_t g;
    st = get_graph(b, K, &g);
    if (st != LBM_OK) return st;
    hipError_t e = hipGraphLaunch(g, b->stream);
    if (e != hipSuccess) return bhip(b, e, "launching the batch graph");
    for (auto &in : b->inst) {
      if (!in.h) continue;
      const int s = int(std::min<int64_t>(K, in.remaining));
      in.h->cur ^= s & 1;
      in.h->step += s;
      in.remaining -= s;
    }
    nsteps -= K;
  }
  return LBM_OK;
}

lbm_status lbm_batch_remaining(const lbm_batch *b, int32_t id, int64_t *remaining) {
  if (!b) return LBM_EINVAL;
  if (!remaining || id < 0 || id >= b->max_inst || !b->inst[id].h)
    return bfail(b, LBM_EINVAL, "unknown simulation id");
  *remaining = b->inst[id].remaining;
  return LBM_OK;
}

lbm_status lbm_batch_read_fields(lbm_batch *b, int32_t id, double *phi, double *psi,
                                 double *ux, double *uy, double *P) {
  if (!b) return LBM_EINVAL;
  if (id < 0 || id >= b->max_inst || !b->inst[id].h)
    return bfail(b, LBM_EINVAL, "unknown simulation id");
  lbm_handle *h = b->inst[id].h;
  lbm_status st = lbm_read_fields(h, phi, psi, ux, uy, P);
  if (st != LBM_OK) bfail(b, st, h->err);
  return st;
}

lbm_status lbm_batch_moments(lbm_batch *b, int32_t id, lbm_moments_t *out) {
  if (!b) return LBM_EINVAL;
  if (id < 0 || id >= b->max_inst || !b->inst[id].h)
    return bfail(b, LBM_EINVAL, "unknown simulation id");
  lbm_handle *h = b->inst[id].h;
  lbm_status st = lbm_moments(h, out);
  if (st != LBM_OK) bfail(b, st, h->err);
  return st;
}

lbm_status lbm_batch_shape(lbm_batch *b, int32_t id, lbm_shape_t *out) {
  if (!b) return LBM_EINVAL;
  if (id < 0 || id >= b->max_inst || !b->inst[id].h)
    return bfail(b, LBM_EINVAL, "unknown simulation id");
  lbm_handle *h = b->inst[id].h;
  lbm_status st = lbm_shape(h, out);
  if (st != LBM_OK) bfail(b, st, h->err);
  return st;
}

lbm_status lbm_batch_retire(lbm_batch *b, int32_t id) {
  if (!b) return LBM_EINVAL;
  if (id < 0 || id >= b->max_inst || !b->inst[id].h)
    return bfail(b, LBM_EINVAL, "unknown simulation id");
  hipError_t e = hipStreamSynchronize(b->stream);  // no launch still uses it
  if (e != hipSuccess) return bhip(b, e, "synchronising");
  auto &in = b->inst[id];
  lbm_destroy(in.h);
  b->arena.release(in.off, in.bytes);
  in = lbm_batch::Inst();
  b->tiles_dirty = true;
  return LBM_OK;
}

size_t lbm_batch_free_bytes(const lbm_batch *b) { return b ? b->arena.largest() : 0; }

lbm_status lbm_batch_set_schedule(lbm_batch *b, const lbm_schedule *s) {
  if (!b) return LBM_EINVAL;
  if (!schedule_ok(s)) return bfail(b, LBM_EINVAL, "schedule out of range");
  b->sched = *s;
  b->tiles_dirty = true;
  return LBM_OK;
}

lbm_status lbm_batch_get_schedule(const lbm_batch *b, lbm_schedule *s) {
  if (!b) return LBM_EINVAL;
  if (!s) return bfail(b, LBM_EINVAL, "s is NULL");
  *s = b->sched;
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, int64_t probe_steps, lbm_schedule *chosen) {
  if (!b) return LBM_EINVAL;
  if (probe_steps < 1) return bfail(b, LBM_EINVAL, "probe_steps < 1");
  const lbm_schedule keep = b->sched;
  std::vector<lbm_schedule> cands;
  for (int rows : {0, 4, 8, 16})
    for (int per_cu : {0, 4, 8, 16})
      cands.push_back(lbm_schedule{rows, per_cu * b->cus, keep.chunk, 0});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return bhip(b, e, "creating events");
  lbm_schedule best = keep;
  double best_t = -1.0;
  lbm_status st = LBM_OK;
  for (const auto &c : cands) {
    b->sched = c;
    b->tiles_dirty = true;
    double work = 0.0;  // site updates in the timed probe
    for (auto &in : b->inst)
      if (in.h)
        work += double(in.h->p.nx) * in.h->p.ny * double(std::min(probe_steps, in.remaining));
    if (work == 0.0) break;
    st = lbm_batch_step(b, std::min<int64_t>(probe_steps, c.chunk));  // builds graphs
    if (st != LBM_OK) break;
    work = 0.0;
    for (auto &in : b->inst)
      if (in.h)
        work += double(in.h->p.nx) * in.h->p.ny * double(std::min(probe_steps, in.remaining));
    if (work == 0.0) break;
    e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) st = lbm_batch_step(b, probe_steps);
    if (e == hipSuccess && st == LBM_OK) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess && st == LBM_OK) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess && st == LBM_OK) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess || st != LBM_OK) break;
    const double t = double(ms) / work;
    if (best_t < 0.0 || t < best_t) {
      best_t = t;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) {
    b->sched = keep;
    b->tiles_dirty = true;
    return bhip(b, e, "timing the autotuner probes");
  }
  if (st != LBM_OK) {
    b->sched = keep;
    b->tiles_dirty = true;
    return st;
  }
  b->sched = best;
  b->tiles_dirty = true;
  if (chosen) *chosen = best;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  clear_graphs(b);
  for (auto &in : b->inst)
    if (in.h) lbm_destroy(in.h);
  for (int p = 0; p < 3; ++p)
    if (b->h_desc[p]) (void)hipHostFree(b->h_desc[p]);
  if (b->h_count) (void)hipHostFree(b->h_count);
  if (b->h_tiles) (void)hipHostFree(b->h_tiles);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->admit) (void)hipStreamDestroy(b->admit);
  delete b;
}

const char *lbm_batch_last_error(const lbm_batch *b) {
  return b ? b->err.c_str() : g_create_error.c_str();
}

}  // extern "C"

#endif  // LBM_F16_PART
