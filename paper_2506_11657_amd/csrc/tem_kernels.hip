// Device kernels for the shared-pole TEM forward path on gfx950 (CDNA4).
//
// Every operator here acts on the node-padded edge layout described in
// tem_internal.h.  The shifted systems (K + s_j M) x_j = f of eq. (rmj) are
// solved in the symmetric scaling y = M^{1/2} x:
//     (A + s_j) y_j = g,   A = M^{-1/2} K M^{-1/2},   g = M^{-1/2} f,
// where K = C^T W C is applied matrix-free: face circulations of the scaled
// field weighted by h_dual / (mu0 * area), then gathered back onto the edges.
#include <hip/hip_ext.h>

#include <cstdint>
#include <tuple>
#include <cstdlib>

#include "tem_internal.h"

namespace tem {

namespace {

constexpr int kWave = 64;

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm keeps the quotient finite for widely scaled operands
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  double r = b.re / b.im, den = b.re * r + b.im;
  return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
// 1/b with the same scaling as Smith's quotient: two real divisions
__device__ __forceinline__ cplx crecip(cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, t = 1.0 / (b.re + b.im * r);
    return {t, -r * t};
  }
  const double r = b.re / b.im, t = 1.0 / (b.re * r + b.im);
  return {r * t, -t};
}
// Complex vectors are stored as double2 (FP64 path) or float2 (complex FP32
// storage of precision 1); arithmetic is always in double.
__device__ __forceinline__ cplx ldv(const double2* p, long long i) {
  const double2 v = p[i];
  return {v.x, v.y};
}
__device__ __forceinline__ cplx ldv(const float2* p, long long i) {
  const float2 v = p[i];
  return {(double)v.x, (double)v.y};
}
__device__ __forceinline__ void stv(double2* p, long long i, cplx v) { p[i] = make_double2(v.re, v.im); }
__device__ __forceinline__ void stv(float2* p, long long i, cplx v) {
  p[i] = make_float2((float)v.re, (float)v.im);
}
// the value a store of v into V storage keeps
__device__ __forceinline__ cplx as_stored(const double2*, cplx v) { return v; }
__device__ __forceinline__ cplx as_stored(const float2*, cplx v) {
  return {(double)(float)v.re, (double)(float)v.im};
}
__device__ __forceinline__ double zero_of(double) { return 0.0; }
__device__ __forceinline__ cplx zero_of(cplx) { return {0.0, 0.0}; }

__device__ __forceinline__ int flat_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }
__device__ __forceinline__ int flat_threads() { return blockDim.x * blockDim.y * blockDim.z; }

// v as held by lane l of the wavefront (l the same in every lane)
__device__ inline double from_lane(double v, int l) {
  const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)bits, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// v of another lane of the same row of 16 lanes, by a DPP control (both
// 32-bit halves moved by the same pattern)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum of v over the 64 lanes of a full wavefront, the same value in every
// lane and in a fixed order: DPP steps inside each row of 16 lanes (pairs,
// quads, then rotations by 4 and 8 lanes), then the four row sums read from
// lanes 0, 16, 32, 48.  Register-to-register moves, no LDS round trips.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x128>(v);  // row_ror:8
  return (from_lane(v, 0) + from_lane(v, 16)) + (from_lane(v, 32) + from_lane(v, 48));
}

// Deterministic block sum (wave sums, then the waves in fixed order);
// the result is valid in thread 0.  lds needs one double per wave.
// The same two reductions for a block of NT threads known at compile time
// (thread index tid): no read of the block size from the dispatch packet.
// block_sum_n leaves the sum in thread 0; block_total_n gives it to every
// thread (each sums the wave totals in the same fixed order).
template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double* lds, int tid) {
  v = wave_sum(v);
  const int lane = tid % kWave, wid = tid / kWave;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int w = 0; w < (NT + kWave - 1) / kWave; ++w) s += lds[w];
  return s;
}
template <int NT>
__device__ __forceinline__ double block_total_n(double v, double* lds, int tid) {
  v = wave_sum(v);
  const int lane = tid % kWave, wid = tid / kWave;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (NT + kWave - 1) / kWave; ++w) s += lds[w];
  return s;
}

__device__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int tid = flat_tid();
  const int lane = tid % kWave, wid = tid / kWave;
  __syncthreads();
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0)
    for (int w = 0; w < (flat_threads() + kWave - 1) / kWave; ++w) s += lds[w];
  return s;
}

// Publish one partial per block; returns true in every thread of the block
// that finished last (which then sees every partial).
__device__ bool publish_partial(double v, double* partials, unsigned int* counter, int bid, int nblocks,
                                int* flag_lds) {
  if (flat_tid() == 0) {
    __hip_atomic_store(partials + bid, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    unsigned int prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    *flag_lds = (prev == (unsigned)(nblocks - 1));
  }
  __syncthreads();
  const bool last = *flag_lds != 0;
  if (last) __threadfence();
  return last;
}

__device__ __forceinline__ long long node_of(const GridArgs& g, int i, int j, int k) {
  return ((long long)k * g.py + j) * g.px + i;
}

// Loads and stores at a 32-bit byte offset from a base pointer: the offset of
// an entry of a 3 nn real field fits (the library refuses grids where
// 3 nn * 8 bytes reaches 2^32), and the address then comes from a scalar base
// plus one 32-bit offset shared by every array of the same layout, with no
// 64-bit address arithmetic per array.
__device__ __forceinline__ double ld_at(const double* __restrict__ base, unsigned off) {
  return *(const double*)((const char*)base + off);
}
__device__ __forceinline__ void st_at(double* __restrict__ base, unsigned off, double v) {
  *(double*)((char*)base + off) = v;
}

// The lumped mass M_e = 1 / (M^-1/2)^2 from the scaling d = M^-1/2 of an edge,
// zero on the boundary edges (d = 0): the weight of the inner products of the
// unscaled seed vectors.  Hardware reciprocal plus one Newton step (a weight
// good to an ulp; a full division is ten dependent instructions).
__device__ __forceinline__ double mass_weight(double d) {
  const double mi = d * d;
  const double r0 = __builtin_amdgcn_rcp(mi);
  const double r1 = fma(fma(-mi, r0, 1.0), r0, r0);
  return d > 0.0 ? r1 : 0.0;
}

// Map a storage-order edge index to (component, node); returns -1 past the end.
__device__ __forceinline__ int storage_to_node(const GridArgs& g, long long e, long long* node) {
  const long long nex = (long long)g.nx * g.py * g.pz;
  const long long ney = (long long)g.px * g.ny * g.pz;
  const long long nez = (long long)g.px * g.py * g.nz;
  if (e < 0) return -1;
  if (e < nex) {
    const int i = (int)(e % g.nx);
    const long long r = e / g.nx;
    *node = node_of(g, i, (int)(r % g.py), (int)(r / g.py));
    return 0;
  }
  e -= nex;
  if (e < ney) {
    const int i = (int)(e % g.px);
    const long long r = e / g.px;
    *node = node_of(g, i, (int)(r % g.ny), (int)(r / g.ny));
    return 1;
  }
  e -= ney;
  if (e < nez) {
    const int i = (int)(e % g.px);
    const long long r = e / g.px;
    *node = node_of(g, i, (int)(r % g.py), (int)(r / g.py));
    return 2;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Stencil tile: K applied to a scaled field, 2.5-D marching in z.
//
// A block owns TX x TY node columns (i, j) and KZ planes starting at plane
// block zb; it outputs the three edges leaving each owned node (owned nodes
// have i < nx, j < ny, k < nz, so all three edges exist).  Shared memory
// holds the scaled field (dinv * value) of two consecutive node planes with a
// one-node halo, and the face fluxes w_f c_f of the current plane with a
// one-node halo on the low side; the fluxes of the plane below, needed only
// at the thread's own node, are carried in registers.
//
// load(v, c) returns the unscaled value of component c at node v (inside
// the grid); emit(v, c, Kp, u) receives (K p')_c and the unscaled value u at
// an owned node.
// ---------------------------------------------------------------------------
template <typename Val, int TX, int TY, int KZ, typename LoadFn, typename EmitFn>
__device__ void stencil_tile(const GridArgs& g, const double* __restrict__ dinv, int zb, LoadFn load, EmitFn emit) {
  __shared__ Val sp[2][3][TY + 2][TX + 2];     // scaled field dinv * u, two planes
  __shared__ Val su[2][3][TY + 2][TX + 2];     // unscaled field u
  __shared__ double sd[2][3][TY + 2][TX + 2];  // dinv
  __shared__ Val phi[3][TY + 1][TX + 1];       // face fluxes of the current plane

  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = tx + TX * ty;
  constexpr int NT = TX * TY;
  constexpr int NF = ((TX + 1) * (TY + 1) + NT - 1) / NT;  // flux entries per thread
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
  const int k0 = zb * KZ;
  const int kend = min(k0 + KZ, g.nz);
  const int i = i0 + tx, j = j0 + ty;
  const bool own = (i < g.nx) && (j < g.ny);

  // per-thread horizontal weights of the flux entries it computes (fixed over the march)
  double fhx[NF], fhy[NF], fwx[NF], fwy[NF], fwz[NF];
  int fgi[NF], fgj[NF];
#pragma unroll
  for (int q = 0; q < NF; ++q) {
    const int e = tid + q * NT;
    const int li = e % (TX + 1), lj = e / (TX + 1);
    const int gi = i0 - 1 + li, gj = j0 - 1 + lj;
    const bool ok = e < (TX + 1) * (TY + 1) && gi >= 0 && gj >= 0 && gi <= g.nx && gj <= g.ny;
    fgi[q] = ok ? gi : -1;
    fgj[q] = gj;
    fhx[q] = ok ? g.h[0][gi] : 0.0;
    fhy[q] = ok ? g.h[1][gj] : 0.0;
    fwx[q] = ok ? g.dw[0][gi] * g.ih[1][gj] : 0.0;  // times 1/hz(k)
    fwy[q] = ok ? g.dw[1][gj] * g.ih[0][gi] : 0.0;  // times 1/hz(k)
    fwz[q] = ok ? g.ih[0][gi] * g.ih[1][gj] : 0.0;  // times dual_z(k)
  }
  const double ohx = own ? g.h[0][i] : 0.0, ohy = own ? g.h[1][j] : 0.0;

  auto load_plane = [&](int kk) {
    const int slot = kk & 1;
    for (int e = tid; e < (TX + 2) * (TY + 2); e += NT) {
      const int li = e % (TX + 2), lj = e / (TX + 2);
      const int gi = i0 - 1 + li, gj = j0 - 1 + lj;
      const bool in = gi >= 0 && gi < g.px && gj >= 0 && gj < g.py && kk >= 0 && kk < g.pz;
      const long long v = in ? node_of(g, gi, gj, kk) : 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double d = in ? dinv[c * g.nn + v] : 0.0;
        const Val u = (d != 0.0) ? load(v, c) : zero_of(Val{});
        sd[slot][c][lj][li] = d;
        su[slot][c][lj][li] = u;
        sp[slot][c][lj][li] = d * u;
      }
    }
  };
  // fluxes of the three faces owned by a node with halo coordinates (li, lj)
  // in plane kk, from its precomputed horizontal factors
  auto fluxes = [&](int q, int kk, int li, int lj, Val& fx, Val& fy, Val& fz) {
    fx = fy = fz = zero_of(Val{});
    if (fgi[q] < 0 || kk < 0 || kk > g.nz) return;
    const int s0 = kk & 1, s1 = (kk + 1) & 1;
    const double hzk = g.h[2][kk], ihz = g.ih[2][kk], dwz = g.dw[2][kk];
    const double hxi = fhx[q], hyj = fhy[q];
    // Fx: +y, +z, -y, -z ; Fy: +z, +x, -z, -x ; Fz: +x, +y, -x, -y
    fx = (fwx[q] * ihz) * (hyj * sp[s0][1][lj][li] + hzk * sp[s0][2][lj + 1][li] - hyj * sp[s1][1][lj][li] - hzk * sp[s0][2][lj][li]);
    fy = (fwy[q] * ihz) * (hzk * sp[s0][2][lj][li] + hxi * sp[s1][0][lj][li] - hzk * sp[s0][2][lj][li + 1] - hxi * sp[s0][0][lj][li]);
    fz = (fwz[q] * dwz) * (hxi * sp[s0][0][lj][li] + hyj * sp[s0][1][lj][li + 1] - hxi * sp[s0][0][lj + 1][li] - hyj * sp[s0][1][lj][li]);
  };
  // fluxes of the own node at plane k0-1 (needed below the first output plane)
  Val fx_prev = zero_of(Val{}), fy_prev = zero_of(Val{});
  load_plane(k0 - 1);
  load_plane(k0);
  __syncthreads();
  if (own && k0 > 0) {
    const int s0 = (k0 - 1) & 1, s1 = k0 & 1, kk = k0 - 1;
    const int li = tx + 1, lj = ty + 1;
    const double hzk = g.h[2][kk], ihz = g.ih[2][kk];
    const double wx = g.dw[0][i] * g.ih[1][j] * ihz, wy = g.dw[1][j] * g.ih[0][i] * ihz;
    fx_prev = wx * (ohy * sp[s0][1][lj][li] + hzk * sp[s0][2][lj + 1][li] - ohy * sp[s1][1][lj][li] - hzk * sp[s0][2][lj][li]);
    fy_prev = wy * (hzk * sp[s0][2][lj][li] + ohx * sp[s1][0][lj][li] - hzk * sp[s0][2][lj][li + 1] - ohx * sp[s0][0][lj][li]);
  }
  __syncthreads();

  for (int kk = k0; kk < kend; ++kk) {
    load_plane(kk + 1);  // overwrites plane kk-1, no longer needed
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NF; ++q) {
      const int e = tid + q * NT;
      if (e < (TX + 1) * (TY + 1)) {
        const int li = e % (TX + 1), lj = e / (TX + 1);
        Val a, b, c;
        fluxes(q, kk, li, lj, a, b, c);
        phi[0][lj][li] = a;
        phi[1][lj][li] = b;
        phi[2][lj][li] = c;
      }
    }
    __syncthreads();
    if (own) {
      const int li = tx + 1, lj = ty + 1;
      const int slot = kk & 1;
      const Val fx = phi[0][lj][li], fy = phi[1][lj][li], fz = phi[2][lj][li];
      // (K p)_Ex = hx (phi_y(k-1) - phi_y + phi_z - phi_z(j-1)), and cyclically
      const Val kpx = ohx * (fy_prev - fy + fz - phi[2][lj - 1][li]);
      const Val kpy = ohy * (phi[2][lj][li - 1] - fz + fx - fx_prev);
      const Val kpz = g.h[2][kk] * (phi[0][lj - 1][li] - fx + fy - phi[1][lj][li - 1]);
      const long long v = node_of(g, i, j, kk);
      emit(v, 0, kpx, su[slot][0][lj][li], sd[slot][0][lj][li]);
      emit(v, 1, kpy, su[slot][1][lj][li], sd[slot][1][lj][li]);
      emit(v, 2, kpz, su[slot][2][lj][li], sd[slot][2][lj][li]);
      fx_prev = fx;
      fy_prev = fy;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Block-3-D stencil tile: all KZ + 2 node planes of a TX x TY tile plus a
// one-node halo are staged at once.  The raw inputs of every staged value are
// fetched into registers first (fetch(v, c) returns them); the caller's pre()
// then runs while those loads are in flight (typically the reduction of the
// previous kernel's partials that yields the recurrence scalars); finally
// combine(raw) forms the value, which is scaled by M^-1/2 into LDS.  The face
// fluxes of KZ + 1 planes are formed in LDS from the 1-D width products, and
// emit(off, (K p')_c, raw, M^-1/2) receives every owned edge.  fetch and emit
// address an entry by its byte offset off = 8 (c nn + node) in a 3 nn field.
//
// Staging order: thread (tx, ty) fetches its own node column (i, j) through
// all KZ + 2 planes, which holds its owned nodes, so their raw values and
// M^-1/2 stay in registers for emit with no second load; each row of a
// plane is one contiguous 64-entry wave access.  The border ring of the
// tile (2 (TX + 2) + 2 TY entries per plane) is spread over all threads.
// ---------------------------------------------------------------------------
// With SCALED = false the staged values are combine(raw) itself (the caller's
// vectors already carry the M^-1/2 scaling) and M^-1/2 is read at the owned
// nodes only.
template <int TX, int TY, int KZ, bool SCALED = true, typename FetchFn, typename PreFn, typename CombineFn,
          typename EmitFn>
__device__ void stencil_block3d(const GridArgs& g, const double* __restrict__ dinv, int bx, int by, int zb, FetchFn fetch, PreFn pre,
                                CombineFn combine, EmitFn emit) {
  constexpr int NP = KZ + 2;                                // planes loaded
  constexpr int NT = TX * TY;
  constexpr int NF = (TX + 1) * (TY + 1);                   // flux entries per plane
  constexpr int NB = 2 * (TX + 2) + 2 * TY;                 // border entries per plane
  constexpr int NBL = (NP * NB + NT - 1) / NT;              // border entries per thread
  using Raw = decltype(fetch(0u));
  __shared__ double sp[NP][3][TY + 2][TX + 2];
  __shared__ double phi[KZ + 1][3][TY + 1][TX + 1];
  // 1-D weights of the block's flux nodes: x (li = 0..TX), y (lj = 0..TY), z (pl = 0..KZ)
  __shared__ double wxh[TX + 1], wxi[TX + 1], wxd[TX + 1];
  __shared__ double wyh[TY + 1], wyi[TY + 1], wyd[TY + 1];
  __shared__ double wzh[KZ + 1], wzi[KZ + 1], wzd[KZ + 1];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = tx + TX * ty;
  const int i0 = bx * TX, j0 = by * TY;
  const int k0 = zb * KZ;
  const int i = i0 + tx, j = j0 + ty;
  const bool own = (i < g.nx) && (j < g.ny);
  // 1. issue every load: the thread's column (planes k0-1 .. k0+KZ), its
  // share of the border ring, the weights
  Raw cr[NP][3];
  double cd[NP][3];
  const bool col = i < g.px && j < g.py;
  const unsigned cstride = 8u * (unsigned)g.nn;  // bytes per component
  unsigned coff[NP];
#pragma unroll
  for (int pl = 0; pl < NP; ++pl) {
    const int kk = k0 - 1 + pl;
    const bool in = col && kk >= 0 && kk < g.pz;
    coff[pl] = in ? 8u * (unsigned)node_of(g, i, j, kk) : 0u;
    const bool ownpl = pl >= 1 && pl <= KZ;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned off = coff[pl] + c * cstride;
      if (SCALED || ownpl) cd[pl][c] = in ? ld_at(dinv, off) : 0.0;
      else cd[pl][c] = 1.0;
      cr[pl][c] = in ? fetch(off) : Raw{};
    }
  }
  Raw br[NBL][3];
  double bd[NBL][3];
  int bpos[NBL];  // (plane, row, column) of the border entry packed as pl * (TY + 2) * (TX + 2) + lj * (TX + 2) + li
#pragma unroll
  for (int m = 0; m < NBL; ++m) {
    const int b = tid + m * NT;
    const int pl = b / NB, rb = b % NB;
    int li, lj;
    if (rb < TX + 2) {  // the low row
      li = rb;
      lj = 0;
    } else if (rb < 2 * (TX + 2)) {  // the high row
      li = rb - (TX + 2);
      lj = TY + 1;
    } else {  // the low and high column of the rows in between
      const int rr = rb - 2 * (TX + 2);
      lj = 1 + (rr >> 1);
      li = (rr & 1) ? TX + 1 : 0;
    }
    bpos[m] = (pl * (TY + 2) + lj) * (TX + 2) + li;
    const int gi = i0 - 1 + li, gj = j0 - 1 + lj, kk = k0 - 1 + pl;
    const bool in = b < NP * NB && gi >= 0 && gi < g.px && gj >= 0 && gj < g.py && kk >= 0 && kk < g.pz;
    const unsigned boff = in ? 8u * (unsigned)node_of(g, gi, gj, kk) : 0u;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const unsigned off = boff + c * cstride;
      bd[m][c] = SCALED ? (in ? ld_at(dinv, off) : 0.0) : 1.0;
      br[m][c] = in ? fetch(off) : Raw{};
    }
  }
  // 1-D weights of the block's flux nodes: entries (TX + 1) + (TY + 1) + (KZ + 1),
  // loaded into registers now, stored to LDS only after pre() (a store would
  // wait for every load issued before it)
  constexpr int NWE = (TX + 1) + (TY + 1) + (KZ + 1);
  constexpr int NW = (NWE + NT - 1) / NT;
  double wv[NW][3];
  // branch-free (selected pointers, clamped index): a load under a branch
  // would be waited for inside it
  bool wok[NW];
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    const int e = tid + m * NT;
    const bool onx = e < TX + 1, ony = !onx && e < (TX + 1) + (TY + 1);
    const int gi = onx ? i0 - 1 + e : ony ? j0 - 1 + (e - (TX + 1)) : k0 - 1 + (e - (TX + 1) - (TY + 1));
    const int hi = onx ? g.nx : ony ? g.ny : g.nz;
    wok[m] = e < NWE && gi >= 0 && gi <= hi;
    // the nine axis arrays are one allocation, axis a at h[0] + 3 a L with
    // h, 1/h and dual widths L apart (a pointer chosen per lane would put the
    // argument block in scratch)
    const long long L = g.ih[0] - g.h[0];
    const double* b = g.h[0] + 3 * (onx ? 0 : ony ? 1 : 2) * L + (wok[m] ? gi : 0);
    wv[m][0] = b[0];
    wv[m][1] = b[L];
    wv[m][2] = b[2 * L];
  }
  // the owner's widths for the edges it emits (clamped for threads that own none)
  const double ohx = g.h[0][min(i, g.nx)], ohy = g.h[1][min(j, g.ny)];
  double ohz[KZ];
#pragma unroll
  for (int z = 0; z < KZ; ++z) ohz[z] = g.h[2][min(k0 + z, g.nz)];
  // 2. the caller's reduction overlaps the loads above
  pre();
#pragma unroll
  for (int m = 0; m < NW; ++m) {
    const int e = tid + m * NT;
    if (!wok[m]) wv[m][0] = wv[m][1] = wv[m][2] = 0.0;
    if (e < TX + 1) {
      wxh[e] = wv[m][0], wxi[e] = wv[m][1], wxd[e] = wv[m][2];
    } else if (e < (TX + 1) + (TY + 1)) {
      const int q = e - (TX + 1);
      wyh[q] = wv[m][0], wyi[q] = wv[m][1], wyd[q] = wv[m][2];
    } else if (e < NWE) {
      const int q = e - (TX + 1) - (TY + 1);
      wzh[q] = wv[m][0], wzi[q] = wv[m][1], wzd[q] = wv[m][2];
    }
  }
  // 3. staged values into LDS
#pragma unroll
  for (int pl = 0; pl < NP; ++pl)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      sp[pl][c][ty + 1][tx + 1] = SCALED ? cd[pl][c] * combine(cr[pl][c]) : combine(cr[pl][c]);
#pragma unroll
  for (int m = 0; m < NBL; ++m)
    if (tid + m * NT < NP * NB) {
      const int pos = bpos[m];
      const int li = pos % (TX + 2), lj = (pos / (TX + 2)) % (TY + 2), pl = pos / ((TX + 2) * (TY + 2));
#pragma unroll
      for (int c = 0; c < 3; ++c) sp[pl][c][lj][li] = SCALED ? bd[m][c] * combine(br[m][c]) : combine(br[m][c]);
    }
  __syncthreads();
  // fluxes of planes k0-1 .. k0+KZ-1 (plane index pl: kk = k0 - 1 + pl)
  for (int e = tid; e < (KZ + 1) * NF; e += NT) {
    const int pl = e / NF, r = e % NF;
    const int li = r % (TX + 1), lj = r / (TX + 1);
    const int gi = i0 - 1 + li, gj = j0 - 1 + lj, kk = k0 - 1 + pl;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (gi >= 0 && gj >= 0 && kk >= 0 && gi <= g.nx && gj <= g.ny && kk <= g.nz) {
      const double hxi = wxh[li], hyj = wyh[lj], hzk = wzh[pl];
      const double wx = wxd[li] * wyi[lj] * wzi[pl];
      const double wy = wyd[lj] * wzi[pl] * wxi[li];
      const double wz = wzd[pl] * wxi[li] * wyi[lj];
      const int a = pl, b = pl + 1;  // planes kk and kk+1 in sp
      fx = wx * (hyj * sp[a][1][lj][li] + hzk * sp[a][2][lj + 1][li] - hyj * sp[b][1][lj][li] - hzk * sp[a][2][lj][li]);
      fy = wy * (hzk * sp[a][2][lj][li] + hxi * sp[b][0][lj][li] - hzk * sp[a][2][lj][li + 1] - hxi * sp[a][0][lj][li]);
      fz = wz * (hxi * sp[a][0][lj][li] + hyj * sp[a][1][lj][li + 1] - hxi * sp[a][0][lj + 1][li] - hyj * sp[a][1][lj][li]);
    }
    phi[pl][0][lj][li] = fx;
    phi[pl][1][lj][li] = fy;
    phi[pl][2][lj][li] = fz;
  }
  __syncthreads();
  if (!own) return;
  const int li = tx + 1, lj = ty + 1;
#pragma unroll
  for (int z = 0; z < KZ; ++z) {
    const int kk = k0 + z;
    if (kk >= g.nz) break;
    const int p = z + 1;  // flux plane of kk, and its column plane
    const double fx = phi[p][0][lj][li], fy = phi[p][1][lj][li], fz = phi[p][2][lj][li];
    const double kpx = ohx * (phi[p - 1][1][lj][li] - fy + fz - phi[p][2][lj - 1][li]);
    const double kpy = ohy * (phi[p][2][lj][li - 1] - fz + fx - phi[p - 1][0][lj][li]);
    const double kpz = ohz[z] * (phi[p][0][lj - 1][li] - fx + fy - phi[p][1][lj][li - 1]);
    emit(coff[p], kpx, cr[p][0], cd[p][0]);
    emit(coff[p] + cstride, kpy, cr[p][1], cd[p][1]);
    emit(coff[p] + 2 * cstride, kpz, cr[p][2], cd[p][2]);
  }
}

constexpr int STX = 32, STY = 4, SKZ = 2;
constexpr int UPD_T = 512;       // threads per block of the seed update and init
constexpr int UPD_BLOCKS = 512;  // blocks of the seed update (= partials it leaves)
constexpr int UPD_PF = 4;        // elements per thread loaded ahead of the update's reduction

// Fixed-order sum of n partials written by the previous kernel (every block
// of the reading kernel computes the same value; no inter-block traffic).

// ---------------------------------------------------------------------------
// Seed CG on A0 = A + s0, iteration k (local = k mod B):
//   stencil: rr_k = sum of the update's partials, beta_{k-1} = rr_k / rr_{k-1};
//            p_k = r_k + beta_{k-1} p_{k-1};  q = A0 p_k;  partials of (p_k, q)
//   update:  alpha_k = rr_k / (p_k, q);  r_{k+1} = r_k - alpha_k q;  partials of (r_{k+1}, r_{k+1})
// Reductions cross kernel boundaries only: a kernel writes one partial per
// block and the next kernel sums them in a fixed order, so results are
// bitwise repeatable and no device-scope fences are needed.
// ---------------------------------------------------------------------------
// One tile of the seed stencil: tile (bx, by, bz) of the grid, block index bid
// among the stencil's nst blocks (its partial-sum slot).  XS (with B3D): the
// vectors are unscaled (M^-1/2 v, as in the one-kernel form): the halo stages
// r and p_old only, the owned edges form q = M^-1 K p + s0 p and the M-weighted
// (p, q); the update then weights (r, r) by M.
template <int TX, int TY, int KZ, bool B3D, bool XS = false>
__device__ __forceinline__ void seed_stencil_tile(const GridArgs& g, const double* __restrict__ r,
                                                  const double* __restrict__ pold, double* __restrict__ pnew,
                                                  double* __restrict__ q, const double* __restrict__ dinv, double s0,
                                                  const double* __restrict__ upd_partials,
                                                  double* __restrict__ partials, SolveState* st, int local, int bx,
                                                  int by, int bz, int bid) {
  constexpr int NT = TX * TY;
  constexpr int NPART = (UPD_BLOCKS + NT - 1) / NT;
  __shared__ double red[(NT + kWave - 1) / kWave];
  const int tid = threadIdx.x + TX * threadIdx.y;
  // requested before the stencil's own loads so that their round trips
  // overlap those loads: the update's partials, rr_{k-1} and the block length
  // (unconditional loads of clamped indices: a load under a branch would be
  // waited for inside it)
  double part[NPART];
#pragma unroll
  for (int m = 0; m < NPART; ++m) part[m] = upd_partials[min(tid + m * NT, UPD_BLOCKS - 1)];
  const double rr_prev = st->rrk[(local + 1) & 1];
  const int B = st->B;
  double beta = 0.0;
  // rr_k from the update's partials, beta_{k-1} = rr_k / rr_{k-1} (rr_{-1} = inf gives 0)
  auto pre = [&]() {
    double sp = tid < UPD_BLOCKS ? part[0] : 0.0;
#pragma unroll
    for (int m = 1; m < NPART; ++m) sp += tid + m * NT < UPD_BLOCKS ? part[m] : 0.0;
    const double rr = block_total_n<NT>(sp, red, tid);
    beta = rr / rr_prev;
    if (bid == 0 && tid == 0) {
      if (isinf(rr_prev)) {  // first iteration: rr_0 = (g, g) scales the stopping tolerance
        st->rr0 = rr;
        st->tol2 *= rr;
      }
      st->rrk[local & 1] = rr;
      const int prev = (local + B - 1) % B;  // the step k-1
      st->beta_h[prev] = beta;
      st->rr_h[prev] = rr;
      if (!isfinite(rr)) st->breakdown = 1;
    }
  };
  double dot = 0.0;
  auto emit = [&](long long v, int c, double kp, double u, double d) {
    const long long e = c * g.nn + v;
    const double out = d * kp + s0 * u;
    pnew[e] = u;
    q[e] = out;
    dot += u * out;
  };
  if constexpr (B3D) {
    struct RP {
      double r, p;
    };
    auto fetch = [&](unsigned off) { return RP{ld_at(r, off), ld_at(pold, off)}; };
    auto combine = [&](const RP& x) { return x.r + beta * x.p; };
    auto emit_raw = [&](unsigned off, double kp, const RP& x, double d) {
      const double u = combine(x);
      const double out = XS ? (d * d) * kp + s0 * u : d * kp + s0 * u;
      st_at(pnew, off, u);
      st_at(q, off, out);
      dot += XS ? mass_weight(d) * u * out : u * out;
    };
    stencil_block3d<TX, TY, KZ, !XS>(g, dinv, bx, by, bz, fetch, pre, combine, emit_raw);
  } else {
    pre();
    auto load = [&](long long v, int c) { return r[c * g.nn + v] + beta * pold[c * g.nn + v]; };
    stencil_tile<double, TX, TY, KZ>(g, dinv, bz, load, emit);
  }
  const double s = block_sum_n<NT>(dot, red, tid);
  if (tid == 0) partials[bid] = s;
}

// 4 waves per SIMD keeps two 512-thread tiles resident per CU (the LDS of
// two tiles fits); the staged registers must then fit in 128 VGPRs
template <int TX, int TY, int KZ, bool B3D, bool XS = false>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(TX * TY * KZ > 512 ? 2 : 4))) k_seed_stencil(GridArgs g, const double* __restrict__ r,
                                                          const double* __restrict__ pold,
                                                          double* __restrict__ pnew, double* __restrict__ q,
                                                          const double* __restrict__ dinv, double s0,
                                                          const double* __restrict__ upd_partials,
                                                          double* __restrict__ partials, SolveState* st, int local) {
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  seed_stencil_tile<TX, TY, KZ, B3D, XS>(g, r, pold, pnew, q, dinv, s0, upd_partials, partials, st, local,
                                         blockIdx.x, blockIdx.y, blockIdx.z, bid);
}

// ---------------------------------------------------------------------------
// Seed CG in one kernel per iteration: the update of step i fused with the
// stencil of step i + 1, with one reduction point between kernels.  Kernel
// `local` (step i = k0 + local of the block starting at k0) reads r_i, p_i and
// q_i = A0 p_i and the partial sums of four inner products of step i, then
//   alpha_i = (r_i, r_i) / (p_i, q_i)
//   (r_{i+1}, r_{i+1}) ~ (r_i, r_i) - 2 alpha_i (r_i, q_i) + alpha_i^2 (q_i, q_i)
//   beta_i = that / (r_i, r_i)
//   r_{i+1} = r_i - alpha_i q_i,  p_{i+1} = r_{i+1} + beta_i p_i,  q_{i+1} = A0 p_{i+1}
// and leaves the partials of (r_{i+1}, r_{i+1}), (p_{i+1}, q_{i+1}),
// (r_{i+1}, q_{i+1}), (q_{i+1}, q_{i+1}).  r_{i+1} and p_{i+1} are formed on
// the tile's halo from r_i, q_i and p_i (three loads per staged entry).
// As in the two-kernel form, q = A0 p is applied to the search direction
// itself, so the residual recurrence carries no rounding amplified by ||A0||
// (the arrangement of Chronopoulos and Gear, which applies A0 to r and keeps
// A0 p by a second recurrence, lost two orders of attainable accuracy on
// these systems); alpha always divides the inner product of the stored
// residual, and only beta uses the one-step expansion, whose cancellation is
// bounded by the residual's reduction in one step.  The recorded history
// (alpha_k, beta_k, (r_{k+1}, r_{k+1}) of the block's steps) and the ring
// (r_{k0+l} in slot l) are those of the two-kernel form, and the history is
// complete after the block's last kernel.
// Buffers ping-pong by parity: kernel `local` reads p, q and partial set
// local & 1 and writes set (local + 1) & 1; set m of the partials holds the
// four inner products at parts + (4 m + v) NS, NS = kReduceSlots.
// With first != 0 the kernel is the prologue of the solve: alpha = beta = 0
// (pass p = q = r), so it forms p_0 = r_0, q_0 = A0 r_0 and the partials of
// step 0 into set 0, and writes no state and no residual.
// XS: the vectors are kept unscaled, v_x = M^-1/2 v (the Jacobi-preconditioned
// CG on K + s0 M, the same iteration): no scaling on the halo, and at owned
// edges q_x = M^-1 (K p_x) + s0 p_x and the inner products weighted by M
// (1 / (M^-1/2)^2, zero on the boundary edges, where every vector is zero).
// The ring then holds M^-1/2 r, which the block update scales back.
template <int NT>
__device__ __forceinline__ void block_total4_n(double v[4], double (*lds)[(NT + kWave - 1) / kWave], int tid) {
#pragma unroll
  for (int m = 0; m < 4; ++m) v[m] = wave_sum(v[m]);
  const int lane = tid % kWave, wid = tid / kWave;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int m = 0; m < 4; ++m) lds[m][wid] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double t = 0.0;
    for (int w = 0; w < (NT + kWave - 1) / kWave; ++w) t += lds[m][w];
    v[m] = t;
  }
}

template <int TX, int TY, int KZ, bool XS>
__device__ __forceinline__ void seed_step_tile(const GridArgs& g, const double* __restrict__ r,
                                               const double* __restrict__ p, const double* __restrict__ q,
                                               double* __restrict__ rn, double* __restrict__ pn,
                                               double* __restrict__ qn, const double* __restrict__ dinv, double s0,
                                               const double* __restrict__ pin, double* __restrict__ pout, int nparts,
                                               SolveState* st, int local, int first, int bx, int by, int bz,
                                               int bid) {
  constexpr int NT = TX * TY;
  constexpr int NW = (NT + kWave - 1) / kWave;
  constexpr int MP = 2;  // partials per thread and product requested ahead of the stencil's loads
  __shared__ double red[4][NW];
  const int tid = threadIdx.x + TX * threadIdx.y;
  double pf[4][MP];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int m = 0; m < MP; ++m) pf[v][m] = pin[v * kReduceSlots + min(tid + m * NT, nparts - 1)];
  const int B = st->B;
  const double carry_a = st->alpha_h[B - 1], carry_b = st->beta_h[B - 1];
  const double rr_sentinel = st->rrk[1];
  double alpha = 0.0, beta = 0.0;
  auto pre = [&]() {
    double t[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      t[v] = 0.0;
#pragma unroll
      for (int m = 0; m < MP; ++m)
        if (tid + m * NT < nparts) t[v] += pf[v][m];
      for (int ix = tid + MP * NT; ix < nparts; ix += NT) t[v] += pin[v * kReduceSlots + ix];
    }
    block_total4_n<NT>(t, red, tid);
    if (first) return;
    const double rr = t[0], pq = t[1], rq = t[2], qq = t[3];
    const bool ok = pq > 0.0 && isfinite(pq);
    alpha = ok ? rr / pq : 0.0;
    const double rr_next = rr - 2.0 * alpha * rq + alpha * alpha * qq;
    const bool ok2 = rr_next >= 0.0 && isfinite(rr_next);
    beta = ok2 ? rr_next / rr : 0.0;
    if (bid == 0 && tid == 0) {
      if (isinf(rr_sentinel)) {  // first step: rr_0 = (g, g) scales the stopping tolerance
        st->rr0 = rr;
        st->tol2 *= rr;
        st->rrk[1] = rr;
      }
      if (local == 0) {  // alpha, beta of the step before this block, for the shift recurrences
        st->carry_alpha = carry_a;
        st->carry_beta = carry_b;
      }
      st->alpha_h[local] = alpha;
      st->beta_h[local] = beta;
      st->rr_h[local] = rr_next;
      st->pAp = pq;
      if (!isfinite(rr) || !ok || !ok2) st->breakdown = 1;
    }
  };
  struct RPQ {
    double r, p, q;
  };
  auto fetch = [&](unsigned off) { return RPQ{ld_at(r, off), ld_at(p, off), ld_at(q, off)}; };
  auto rnext = [&](const RPQ& x) { return x.r - alpha * x.q; };
  auto combine = [&](const RPQ& x) { return rnext(x) + beta * x.p; };
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto emit = [&](unsigned off, double kp, const RPQ& x, double d) {
    const double rv = rnext(x);
    const double pv = combine(x);
    if (!first) st_at(rn, off, rv);
    st_at(pn, off, pv);
    if constexpr (XS) {
      const double qv = (d * d) * kp + s0 * pv;
      const double mq = mass_weight(d) * qv;
      st_at(qn, off, qv);
      acc[0] += mass_weight(d) * rv * rv;
      acc[1] += pv * mq;
      acc[2] += rv * mq;
      acc[3] += qv * mq;
    } else {
      const double qv = d * kp + s0 * pv;
      st_at(qn, off, qv);
      acc[0] += rv * rv;
      acc[1] += pv * qv;
      acc[2] += rv * qv;
      acc[3] += qv * qv;
    }
  };
  stencil_block3d<TX, TY, KZ, !XS>(g, dinv, bx, by, bz, fetch, pre, combine, emit);
  // fixed-order block sums of the four products
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = wave_sum(acc[m]);
  const int lane = tid % kWave, wid = tid / kWave;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int m = 0; m < 4; ++m) red[m][wid] = acc[m];
  __syncthreads();
  if (tid < 4) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[tid][w];
    pout[tid * kReduceSlots + bid] = t;
  }
}

// three staged vectors need more than the 128 VGPRs of 4 waves per SIMD
template <int TX, int TY, int KZ, bool XS>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(2)))
k_seed_step(GridArgs g, const double* __restrict__ r, const double* __restrict__ p, const double* __restrict__ q,
            double* __restrict__ rn, double* __restrict__ pn, double* __restrict__ qn, const double* __restrict__ dinv,
            double s0, const double* __restrict__ pin, double* __restrict__ pout, SolveState* st, int local,
            int first) {
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int nparts = gridDim.x * gridDim.y * gridDim.z;
  seed_step_tile<TX, TY, KZ, XS>(g, r, p, q, rn, pn, qn, dinv, s0, pin, pout, nparts, st, local, first, blockIdx.x,
                                 blockIdx.y, blockIdx.z, bid);
}

// Block blk of the nblk blocks of one seed update (grid-stride over the n entries).
// wd != nullptr: unscaled vectors, (r, r) weighted by M from wd = M^-1/2.
__device__ __forceinline__ void seed_update_block(long long n, const double* __restrict__ r,
                                                  const double* __restrict__ q, double* __restrict__ rnext,
                                                  const double* __restrict__ st_partials, int n_st,
                                                  double* __restrict__ partials, SolveState* st, int local, int blk,
                                                  int nblk, const double* __restrict__ wd) {
  __shared__ double red[UPD_T / 64];
  const int tid = threadIdx.x;
  // requested first, so that their round trips overlap the loads of r and q
  // below: this thread's first stencil partial (clamped index, no branch),
  // rr_k and B
  const double part0 = st_partials[min(tid, n_st - 1)];
  const double rr = st->rrk[local & 1];
  const int B = st->B;
  // the first UPD_PF grid-stride elements are loaded before the reduction so
  // that their latency overlaps the sum of the stencil's partials
  const long long stride = (long long)nblk * UPD_T;
  const long long e0 = blk * (long long)UPD_T + tid;
  double rv[UPD_PF], qv[UPD_PF], dv[UPD_PF];
#pragma unroll
  for (int m = 0; m < UPD_PF; ++m) {
    const long long e = e0 + m * stride;
    rv[m] = e < n ? r[e] : 0.0;
    qv[m] = e < n ? q[e] : 0.0;
    dv[m] = (wd && e < n) ? wd[e] : 1.0;
  }
  // fixed-order sum: this thread's partials in index order, then the block
  double sp = tid < n_st ? part0 : 0.0;
  for (int i = tid + UPD_T; i < n_st; i += UPD_T) sp += st_partials[i];
  const double pap = block_total_n<UPD_T>(sp, red, tid);
  const double alpha = (pap > 0.0 && isfinite(pap)) ? rr / pap : 0.0;
  if (blk == 0 && tid == 0) {
    if (!(pap > 0.0 && isfinite(pap))) st->breakdown = 1;
    if (local == 0) {  // alpha, beta of the step before this block, for the shift recurrences
      st->carry_alpha = st->alpha_h[B - 1];
      st->carry_beta = st->beta_h[B - 1];
    }
    st->alpha_h[local] = alpha;
    st->pAp = pap;
  }
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < UPD_PF; ++m) {
    const long long e = e0 + m * stride;
    if (e < n) {
      const double v = rv[m] - alpha * qv[m];
      rnext[e] = v;
      acc += (wd ? mass_weight(dv[m]) : 1.0) * v * v;
    }
  }
  for (long long e = e0 + UPD_PF * stride; e < n; e += stride) {
    const double v = r[e] - alpha * q[e];
    rnext[e] = v;
    acc += (wd ? mass_weight(wd[e]) : 1.0) * v * v;
  }
  const double s = block_sum_n<UPD_T>(acc, red, tid);
  if (tid == 0) partials[blk] = s;
}

__global__ void __launch_bounds__(UPD_T) k_seed_update(long long n, const double* __restrict__ r,
                                                       const double* __restrict__ q, double* __restrict__ rnext,
                                                       const double* __restrict__ st_partials, int n_st,
                                                       double* __restrict__ partials, SolveState* st, int local,
                                                       const double* __restrict__ wd) {
  seed_update_block(n, r, q, rnext, st_partials, n_st, partials, st, local, blockIdx.x, gridDim.x, wd);
}

// Per-shift recurrences for one block of B seed steps, replayed from the
// recorded alpha_k, beta_k, (r_{k+1}, r_{k+1}); one wavefront per shift, lane l
// owning the coefficients of residual slot l.  For system (A0 + sig) y = g:
//   zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1} /
//                (a_k b_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + sig a_k)),
//   alpha^s_k = a_k zeta_{k+1}/zeta_k,  beta^s_k = b_k (zeta_{k+1}/zeta_k)^2,
//   y_{k+1} = y_k + alpha^s_k p_k,  p_{k+1} = zeta_{k+1} r_{k+1} + beta^s_k p_k,
// accumulated as coefficients of the block's starting p and residuals r_l.
// rr_partials: the n partial sums of (r_{k+1}, r_{k+1}) the block's last seed
// update left, from which the block's last beta_k and (r_{k+1}, r_{k+1}) are
// completed here; n = 0: the seed kernels recorded the whole history.
__device__ __forceinline__ void shift_block_wave(const double* __restrict__ rr_partials, int n, SolveState* st, int j,
                                                 int f) {
  const int lane = threadIdx.x;
  constexpr int NPART = 32;  // partials prefetched per lane (n <= 2048 in one round trip)
  __shared__ double red[1];
  // the partials and the state's scalars are all requested before any is
  // used (one round trip instead of several in sequence)
  double part[NPART];
#pragma unroll
  for (int m = 0; m < NPART; ++m) part[m] = n > 0 ? rr_partials[min(lane + m * kWave, n - 1)] : 0.0;
  const int B = st->B;
  const int is_active = st->active[j];
  // the block's last step: (r_{k+1}, r_{k+1}) from the partials, beta_k
  double sp = 0.0;
#pragma unroll
  for (int m = 0; m < NPART; ++m) sp += lane + m * kWave < n ? part[m] : 0.0;
  for (int m = lane + NPART * kWave; m < n; m += kWave) sp += rr_partials[m];
  const double rr_sum = block_total_n<kWave>(sp, red, lane);
  const double rr_last = n > 0 ? rr_sum : st->rr_h[B - 1];
  const double beta_last = n > 0 ? rr_last / st->rrk[(B - 1) & 1] : st->beta_h[B - 1];
  if (j == 0 && lane == 0) {
    if (n > 0) {
      st->beta_h[B - 1] = beta_last;
      st->rr_h[B - 1] = rr_last;
    }
    st->k += B;
  }
  if (!is_active) {
    if (lane == 0) st->apply[f][j] = 0;
    return;
  }
  const double tol2 = st->tol2;
  const cplx sig{st->sig_re[j], st->sig_im[j]};
  cplx z{st->z_re[j], st->z_im[j]}, zp{st->zp_re[j], st->zp_im[j]};
  cplx a{1.0, 0.0}, c{0.0, 0.0}, e{0.0, 0.0}, d{0.0, 0.0};
  int iters = st->iters[j];
  bool active = true, bad = false;
  double est = st->est[j];
  // the block's history, slot `lane` in lane `lane`, fetched in one round
  // trip; each step below takes its scalars from a lane instead of waiting on
  // memory (the state was written by other kernels, so every such read would
  // miss the caches)
  const double h_alpha = lane < B ? st->alpha_h[lane] : 0.0;
  const double h_beta = lane < B - 1 ? st->beta_h[lane] : beta_last;
  const double h_rr = lane < B - 1 ? st->rr_h[lane] : rr_last;
  const double carry_alpha = st->carry_alpha, carry_beta = st->carry_beta;
  for (int i = 0; i < B && active; ++i) {
    const double a_k = from_lane(h_alpha, i);
    const double b_k = from_lane(h_beta, i);
    const double rr_next = from_lane(h_rr, i);
    const double a_km1 = i ? from_lane(h_alpha, i - 1) : carry_alpha;
    const double b_km1 = i ? from_lane(h_beta, i - 1) : carry_beta;
    const cplx num = a_km1 * cmul(z, zp);
    const cplx one_sa{1.0 + sig.re * a_k, sig.im * a_k};
    const cplx den = (a_k * b_km1) * (zp - z) + a_km1 * cmul(zp, one_sa);
    // zeta_{k+1} / zeta_k = a_{k-1} zeta_{k-1} / den: one reciprocal serves both
    // (divisions are the longest latency chain of this single-wave recurrence)
    const cplx inv = crecip(den);
    const cplx zn = cmul(num, inv);
    const cplx ratio = a_km1 * cmul(zp, inv);
    const cplx as = a_k * ratio;
    const cplx bs = b_k * cmul(ratio, ratio);
    if (!(isfinite(zn.re) && isfinite(zn.im) && isfinite(as.re) && isfinite(as.im) && isfinite(bs.re) &&
          isfinite(bs.im))) {
      bad = true;
      break;
    }
    c = c + cmul(as, a);
    d = d + cmul(as, e);
    e = cmul(bs, e);
    a = cmul(bs, a);
    if (lane == (i + 1) % B) e = zn;
    zp = z;
    z = zn;
    ++iters;
    const double est2 = (zn.re * zn.re + zn.im * zn.im) * rr_next;
    est = sqrt(est2);
    if (est2 <= tol2) active = false;
  }
  if (lane < B) {
    double* cl = st->cf[f][j][1 + lane];
    cl[0] = e.re;
    cl[1] = e.im;
    cl[2] = d.re;
    cl[3] = d.im;
  }
  if (lane == 0) {
    st->apply[f][j] = 1;
    double* c0 = st->cf[f][j][0];
    c0[0] = a.re;
    c0[1] = a.im;
    c0[2] = c.re;
    c0[3] = c.im;
    st->z_re[j] = z.re;
    st->z_im[j] = z.im;
    st->zp_re[j] = zp.re;
    st->zp_im[j] = zp.im;
    st->iters[j] = iters;
    st->est[j] = est;
    st->active[j] = active && !bad;
    if (bad) st->breakdown = 1;
  }
}

__global__ void __launch_bounds__(64) k_shift_block(const double* __restrict__ rr_partials, int n, SolveState* st,
                                                    int f) {
  shift_block_wave(rr_partials, n, st, blockIdx.x, f);
}

// Deferred shift update after a block of BB seed iterations:
//   p_j <- a_j p_j + sum_l e_jl r_l,   y_j <- y_j + c_j p_j + sum_l d_jl r_l
// for every shift updated in the block (coefficients from k_shift_block).
// y_j is stored in YV and p_j in PV: double2 both for the FP64 path, double2
// and float2 for precision 1 (the iterate accumulates in FP64, only the
// search direction is rounded to FP32 once per block).
// The coefficients are the same for every thread, so they are read with
// uniform loads from the state (scalar registers as FMA operands) rather than
// staged through LDS, whose broadcast reads stalled the waves; the kernel
// writes nothing the coefficients could alias.
constexpr int BU_T = 256;
template <int BB, typename YV, typename PV>
__device__ __forceinline__ void block_update_block(long long n3, const double* __restrict__ R,
                                                  const double* __restrict__ R0, YV* __restrict__ Y,
                                                  PV* __restrict__ P, int J, const SolveState* __restrict__ st,
                                                  int f, int blk, int nblk, const double* __restrict__ rscale) {
  for (long long e = blk * (long long)BU_T + threadIdx.x; e < n3; e += (long long)nblk * BU_T) {
    double rl[BB];
    rl[0] = R0[e];
#pragma unroll
    for (int l = 1; l < BB; ++l) rl[l] = R[(long long)l * n3 + e];
    if (rscale) {  // a ring of M^-1/2 r: back to the scaled residuals
      const double sc = rscale[e];
#pragma unroll
      for (int l = 0; l < BB; ++l) rl[l] *= sc;
    }
    for (int j = 0; j < J; ++j) {
      if (!st->apply[f][j]) continue;
      const double* c = st->cf[f][j][0];
      const cplx p = ldv(P, (long long)j * n3 + e);
      const cplx y = ldv(Y, (long long)j * n3 + e);
      double pr = c[0] * p.re - c[1] * p.im;
      double pi = c[0] * p.im + c[1] * p.re;
      double yr = y.re + c[2] * p.re - c[3] * p.im;
      double yi = y.im + c[2] * p.im + c[3] * p.re;
#pragma unroll
      for (int l = 0; l < BB; ++l) {
        const double* cl = c + 4 * (l + 1);
        pr += cl[0] * rl[l];
        pi += cl[1] * rl[l];
        yr += cl[2] * rl[l];
        yi += cl[3] * rl[l];
      }
      stv(P, (long long)j * n3 + e, cplx{pr, pi});
      stv(Y, (long long)j * n3 + e, cplx{yr, yi});
    }
  }
}

template <int BB, typename YV, typename PV>
__global__ void __launch_bounds__(BU_T) k_block_update(long long n3, const double* __restrict__ R,
                                                       const double* __restrict__ R0, YV* __restrict__ Y,
                                                       PV* __restrict__ P, int J,
                                                       const SolveState* __restrict__ st, int f,
                                                       const double* __restrict__ rscale) {
  block_update_block<BB, YV, PV>(n3, R, R0, Y, P, J, st, f, blockIdx.x, gridDim.x, rscale);
}

// ---------------------------------------------------------------------------
// Batched launches: the same per-tile / per-block work as the kernels above for
// several independent multi-shift solves (jobs) at once, one grid per kernel,
// each block finding its job in a device table.  A job's tile decomposition,
// reductions and their order are those of the job run alone in the same
// batched form, so its results do not depend on the other jobs.
// ---------------------------------------------------------------------------
constexpr int kBTX = 64, kBTY = 8, kBKZ = 1;

__global__ void __launch_bounds__(kBTX* kBTY) __attribute__((amdgpu_waves_per_eu(4)))
k_seed_stencil_batch(const BatchJob* __restrict__ jobs, int njobs, int B, int local) {
  int j = 0;
  while (j + 1 < njobs && (int)blockIdx.x >= jobs[j + 1].tile0) ++j;
  const BatchJob& jb = jobs[j];
  const long long n3 = 3 * jb.g.nn;
  const int t = (int)blockIdx.x - jb.tile0;
  const int bx = t % jb.ntx, by = (t / jb.ntx) % jb.nty, bz = t / (jb.ntx * jb.nty);
  seed_stencil_tile<kBTX, kBTY, kBKZ, true>(jb.g, jb.R + (long long)local * n3, jb.pbuf + ((local + 1) & 1) * n3,
                                            jb.pbuf + (local & 1) * n3, jb.q, jb.dinv, jb.s0, jb.part_up, jb.part_st,
                                            jb.st, local, bx, by, bz, t);
}

__global__ void __launch_bounds__(UPD_T) k_seed_update_batch(const BatchJob* __restrict__ jobs, int B, int local) {
  const BatchJob& jb = jobs[blockIdx.x / UPD_BLOCKS];
  const long long n3 = 3 * jb.g.nn;
  seed_update_block(n3, jb.R + (long long)local * n3, jb.q, jb.R + (long long)((local + 1) % B) * n3, jb.part_st,
                    jb.ntiles, jb.part_up, jb.st, local, blockIdx.x % UPD_BLOCKS, UPD_BLOCKS, nullptr);
}

__global__ void __launch_bounds__(64) k_shift_block_batch(const BatchJob* __restrict__ jobs) {
  const BatchJob& jb = jobs[blockIdx.y];
  if ((int)blockIdx.x >= jb.J) return;
  shift_block_wave(jb.part_up, UPD_BLOCKS, jb.st, blockIdx.x, 0);
}

template <int BB>
__global__ void __launch_bounds__(BU_T) k_block_update_batch(const BatchJob* __restrict__ jobs, int njobs) {
  int j = 0;
  while (j + 1 < njobs && (int)blockIdx.x >= jobs[j + 1].bu0) ++j;
  const BatchJob& jb = jobs[j];
  block_update_block<BB, double2, double2>(3 * jb.g.nn, jb.R, jb.R, jb.Y, jb.P, jb.J, jb.st, 0,
                                           (int)blockIdx.x - jb.bu0, jb.nbu, nullptr);
}

// the leading SolveHead of every job's state, contiguous, for one copy to the host
__global__ void k_gather_heads(const BatchJob* __restrict__ jobs, int njobs, SolveHead* out) {
  if ((int)blockIdx.x >= njobs) return;
  const int* src = (const int*)jobs[blockIdx.x].st;
  int* dst = (int*)(out + blockIdx.x);
  for (int i = threadIdx.x; i < (int)(sizeof(SolveHead) / sizeof(int)); i += blockDim.x) dst[i] = src[i];
}

template <typename YV, typename PV>
__global__ void __launch_bounds__(UPD_T) k_seed_init(long long n3, const double* __restrict__ gv, double* r0,
                                                     double* pold, YV* Y, PV* P, int J,
                                                     double* __restrict__ partials, SolveState* st,
                                                     const double* __restrict__ r0_scale) {
  __shared__ double red[UPD_T / 64];
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)gridDim.x * blockDim.x) {
    const double v = gv[e];
    r0[e] = r0_scale ? r0_scale[e] * v : v;  // the residual ring of the unscaled seed form holds M^-1/2 r
    pold[e] = 0.0;
    for (int j = 0; j < J; ++j) {
      stv(Y, (long long)j * n3 + e, cplx{0.0, 0.0});
      stv(P, (long long)j * n3 + e, cplx{v, 0.0});
    }
    acc += v * v;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rrk[1] = INFINITY;          // rr_{-1}: beta_{-1} = 0, so p_0 = r_0
    st->alpha_h[st->B - 1] = 1.0;   // alpha_{-1}
    st->beta_h[st->B - 1] = 0.0;    // beta_{-1}
    st->k = 0;
    st->breakdown = 0;
  }
}

// ---------------------------------------------------------------------------
// Complex shifted operator on nvec vectors, vector index = blockIdx.z / zblocks:
//   out_j = rhs - (A + s_j) X_j   (rhs != nullptr)   or   out_j = (A + s_j) X_j,
// plus per-block partial sums of |out_j|^2 in norm_partials[j * nblocks + b].
// ---------------------------------------------------------------------------
constexpr int CTX = 32, CTY = 4, CKZ = 2;
__global__ void __launch_bounds__(CTX* CTY) k_cstencil(GridArgs g, const double2* __restrict__ X, long long xstride,
                                                       const double* __restrict__ dinv, const double* sre,
                                                       const double* sim, const double2* __restrict__ rhs,
                                                       double2* __restrict__ out, long long ostride,
                                                       double* norm_partials, int zblocks) {
  __shared__ double red[16];
  const int vec = blockIdx.z / zblocks;
  const int zb = blockIdx.z % zblocks;
  const double2* x = X + vec * xstride;
  double2* o = out + vec * ostride;
  const double shr = sre[vec], shi = sim[vec];
  double acc = 0.0;
  auto load = [&](long long v, int c) {
    const double2 t = x[c * g.nn + v];
    return cplx{t.x, t.y};
  };
  auto emit = [&](long long v, int c, cplx kp, cplx uu, double d) {
    const long long e = c * g.nn + v;
    cplx res{0.0, 0.0};
    if (d != 0.0) {
      const double2 u = make_double2(uu.re, uu.im);
      res = cplx{d * kp.re + shr * u.x - shi * u.y, d * kp.im + shr * u.y + shi * u.x};
      if (rhs != nullptr) {
        const double2 b = rhs[e];
        res = cplx{b.x - res.re, b.y - res.im};
      }
    }
    o[e] = make_double2(res.re, res.im);
    acc += res.re * res.re + res.im * res.im;
  };
  stencil_tile<cplx, CTX, CTY, CKZ>(g, dinv, zb, load, emit);
  const int nb = gridDim.x * gridDim.y * zblocks;
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * zb);
  const double s = block_sum(acc, red);
  if (flat_tid() == 0 && norm_partials != nullptr) norm_partials[(long long)vec * nb + bid] = s;
}

__global__ void k_reduce_rows(const double* partials, int cols, double* out) {
  __shared__ double red[8];
  const double* p = partials + (long long)blockIdx.x * cols;
  double s = 0.0;
  for (int i = threadIdx.x; i < cols; i += blockDim.x) s += p[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Operator set-up: lumped mass M_e = 1/4 sum over the four cells touching the
// edge of sigma_c V_c (Sec. 2.2, [M]_ij = (sigma Phi_j, Phi_i) with mass
// lumping) and dinv = M^-1/2 on interior edges (0 on PEC and padding edges).
// ---------------------------------------------------------------------------
__global__ void k_mass(GridArgs g, const double* __restrict__ sigma, double* mass, double* dinv, double* sqrtm) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= g.nn) return;
  const int i = (int)(v % g.px);
  const int j = (int)((v / g.px) % g.py);
  const int k = (int)(v / ((long long)g.px * g.py));
  auto sv = [&](int ci, int cj, int ck) {
    return sigma[((long long)ck * g.ny + cj) * g.nx + ci] * g.h[0][ci] * g.h[1][cj] * g.h[2][ck];
  };
  double m[3] = {0.0, 0.0, 0.0};
  bool in[3];
  in[0] = i < g.nx && j > 0 && j < g.ny && k > 0 && k < g.nz;
  in[1] = j < g.ny && i > 0 && i < g.nx && k > 0 && k < g.nz;
  in[2] = k < g.nz && i > 0 && i < g.nx && j > 0 && j < g.ny;
  if (in[0]) m[0] = 0.25 * (sv(i, j - 1, k - 1) + sv(i, j, k - 1) + sv(i, j - 1, k) + sv(i, j, k));
  if (in[1]) m[1] = 0.25 * (sv(i - 1, j, k - 1) + sv(i, j, k - 1) + sv(i - 1, j, k) + sv(i, j, k));
  if (in[2]) m[2] = 0.25 * (sv(i - 1, j - 1, k) + sv(i, j - 1, k) + sv(i - 1, j, k) + sv(i, j, k));
  for (int c = 0; c < 3; ++c) {
    mass[c * g.nn + v] = m[c];
    dinv[c * g.nn + v] = in[c] ? 1.0 / sqrt(m[c]) : 0.0;
    sqrtm[c * g.nn + v] = in[c] ? sqrt(m[c]) : 0.0;
  }
}

__global__ void k_scale(long long n, const double* a, const double* x, double* y) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e < n) y[e] = a[e] * x[e];
}

// y[e] = 0 for e < n (a fill kernel rather than a memset, so that callers
// may put it in a graph)
__global__ void k_zero2(long long n, double2* y) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e < n) y[e] = make_double2(0.0, 0.0);
}

// p[0] = a, p[1] = b (one thread): scalars placed in device memory by the
// stream itself, with no host staging buffer
__global__ void k_store2(double* p, double a, double b) {
  if (threadIdx.x == 0) {
    p[0] = a;
    p[1] = b;
  }
}

__global__ void k_to_complex(long long n, const double* x, double2* y) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e < n) y[e] = make_double2(x[e], 0.0);
}

// ---------------------------------------------------------------------------
// Residue contraction (Sec. 3.2, the product S R): fields in storage order,
//   U[k][e] = dinv_e * sum_j Re(C_jk Y_j[e]) = [Re Y | Im Y] [Re C ; -Im C],
// as an (edges x 2J) x (2J x T) product on FP64 MFMA (v_mfma_f64_16x16x4f64).
// One wave computes 16 edges x all channels (T <= 64).
// Lane layout of the 16x16x4 FP64 MFMA (checked on the device): lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and its result register r holds
// D[4*r + l/16][l%16], r = 0..3.
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_contract(GridArgs g, const double2* __restrict__ Y, int J,
                                                  const double* __restrict__ dinv, const double* __restrict__ C,
                                                  int T, double* __restrict__ U, long long nstore) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long e0 = ((long long)blockIdx.x * 4 + wave) * 16;
  const int row = lane & 15, kq = lane >> 4;
  long long node = 0;
  const long long ea = e0 + row;
  const int comp = ea < nstore ? storage_to_node(g, ea, &node) : -1;
  const double dv = comp >= 0 ? dinv[comp * g.nn + node] : 0.0;
  const int K2 = 2 * J;
  const int nT = (T + 15) / 16;
  d4 acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int kb = 0; kb < K2; kb += 4) {
    const int kk = kb + kq;
    double a = 0.0;
    if (kk < K2 && comp >= 0 && dv != 0.0) {
      const double2 yv = Y[(long long)(kk >> 1) * 3 * g.nn + comp * g.nn + node];
      a = dv * ((kk & 1) ? yv.y : yv.x);
    }
    for (int t = 0; t < nT; ++t) {
      const int ch = t * 16 + row;
      double b = 0.0;
      if (kk < K2 && ch < T) {
        const double* cc = C + 2 * ((long long)(kk >> 1) * T + ch);
        b = (kk & 1) ? -cc[1] : cc[0];
      }
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
  for (int t = 0; t < nT; ++t) {
    const int ch = t * 16 + row;
    if (ch >= T) continue;
    for (int r = 0; r < 4; ++r) {
      const long long e = e0 + 4 * r + kq;
      if (e < nstore) U[(long long)ch * nstore + e] = acc[t][r];
    }
  }
}

// Receivers: z_jr = sum over the 4 edges of the surface z-face of
// q_e dinv_e Y_j[e] with q = -(circulation)/(area) (dB_z/dt = -(curl e)_z),
// then d[k][r] = Re sum_j C_jk z_jr.  One thread per (channel, receiver).
__global__ void k_receivers(GridArgs g, const double2* __restrict__ Y, int J, const double* __restrict__ dinv,
                            const double* __restrict__ C, int T, const int* __restrict__ rx, int n_rx, int ks,
                            double* d) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= T * n_rx) return;
  const int ch = idx / n_rx, r = idx % n_rx;
  const int i = rx[2 * r], j = rx[2 * r + 1];
  const double hx = g.h[0][i], hy = g.h[1][j];
  const double inva = -1.0 / (hx * hy);
  const long long e[4] = {0 * g.nn + node_of(g, i, j, ks), 1 * g.nn + node_of(g, i + 1, j, ks),
                          0 * g.nn + node_of(g, i, j + 1, ks), 1 * g.nn + node_of(g, i, j, ks)};
  const double w[4] = {hx * inva, hy * inva, -hx * inva, -hy * inva};
  double acc = 0.0;
  for (int jj = 0; jj < J; ++jj) {
    double zr = 0.0, zi = 0.0;
    for (int m = 0; m < 4; ++m) {
      const double2 yv = Y[(long long)jj * 3 * g.nn + e[m]];
      const double s = w[m] * dinv[e[m]];
      zr += s * yv.x;
      zi += s * yv.y;
    }
    const double* cc = C + 2 * ((long long)jj * T + ch);
    acc += cc[0] * zr - cc[1] * zi;
  }
  d[(long long)ch * n_rx + r] = acc;
}

// ---------------------------------------------------------------------------
// Two-pass form (no per-shift vectors).  Every shifted iterate is a fixed
// combination of the seed residuals, y_j = sum_k gamma_jk r_k, and so is every
// channel, u(t) = sum_k r_k w_kt with w_kt = Re sum_j c_jt gamma_jk (the host
// derives gamma from the seed's recorded alpha_k, beta_k).  The kernels below
// read the residuals a block leaves in its ring: after the block whose first
// iteration is k0, slot l holds r_{k0+l} for l = 1 .. B-1 and slot 0 holds
// r_{k0+B}; r_0 = g sits in slot 0 before the first block.
// ---------------------------------------------------------------------------

// q_r . (M^-1/2 r_k) for the block's residuals (init: r_0 only), into
// hq[(l - 1) * n_rx + r] (init: hq[r]); receiver rows as in k_receivers.
__global__ void k_ring_receivers(GridArgs g, const double* __restrict__ R, int B, const double* __restrict__ dinv,
                                 const int* __restrict__ rx, int n_rx, int ks, double* hq, int init) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int nl = init ? 1 : B;
  if (idx >= nl * n_rx) return;
  const int l = init ? 0 : idx / n_rx + 1;
  const int r = idx % n_rx;
  const double* rv = R + (long long)(l % B) * 3 * g.nn;
  const int i = rx[2 * r], j = rx[2 * r + 1];
  const double hx = g.h[0][i], hy = g.h[1][j];
  const double inva = -1.0 / (hx * hy);
  const long long e[4] = {0 * g.nn + node_of(g, i, j, ks), 1 * g.nn + node_of(g, i + 1, j, ks),
                          0 * g.nn + node_of(g, i, j + 1, ks), 1 * g.nn + node_of(g, i, j, ks)};
  const double w[4] = {hx * inva, hy * inva, -hx * inva, -hy * inva};
  double acc = 0.0;
  for (int m = 0; m < 4; ++m) acc += w[m] * (dinv ? dinv[e[m]] : 1.0) * rv[e[m]];
  hq[idx] = acc;
}

// U[t][e] = r_0[e] W[0][t] (padded layout, channel-major): the first term.
__global__ void k_ring_contract_init(long long n3, const double* __restrict__ r0, const double* __restrict__ W,
                                     int T, double* U) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const double v = r0[e];
  for (int t = 0; t < T; ++t) U[(long long)t * n3 + e] = v * W[t];
}

// U[t][e] += sum_{l=1..B} r_{k0+l}[e] W[k0+l][t] for the block just finished
// (k0 = st->k - B): an (entries x B) x (B x T) product on FP64 MFMA
// (v_mfma_f64_16x16x4f64, lane layout as in k_contract), one wave per 16
// entries and all T <= 64 channels.
__global__ void __launch_bounds__(256) k_ring_contract(long long n3, const double* __restrict__ R, int B,
                                                       const double* __restrict__ W, int T, double* U,
                                                       const SolveState* __restrict__ st) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long e0 = ((long long)blockIdx.x * 4 + wave) * 16;
  const int row = lane & 15, kq = lane >> 4;
  const long long ea = e0 + row;
  const long long k0 = (long long)st->k - B;
  const int nT = (T + 15) / 16;
  d4 acc[4];
  for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int lb = 0; lb < B; lb += 4) {
    const int l = lb + kq + 1;  // residual r_{k0+l}, l = 1 .. B
    const double a = (l <= B && ea < n3) ? R[(long long)(l % B) * n3 + ea] : 0.0;
    for (int t = 0; t < nT; ++t) {
      const int ch = t * 16 + row;
      const double b = (l <= B && ch < T) ? W[(k0 + l) * T + ch] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
  for (int t = 0; t < nT; ++t) {
    const int ch = t * 16 + row;
    if (ch >= T) continue;
    for (int r = 0; r < 4; ++r) {
      const long long e = e0 + 4 * r + kq;
      if (e < n3) U[(long long)ch * n3 + e] += acc[t][r];
    }
  }
}

// fields[t][e] = dinv_e U[t][node(e)] in storage order, and the receivers
// d[t][r] = q_r . (M^-1/2 U[t]) (one thread per (channel, receiver) after the
// fields, in a second launch)
__global__ void k_ring_fields(GridArgs g, const double* __restrict__ U, int T, const double* __restrict__ dinv,
                              double* fields, long long nstore) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= nstore) return;
  long long node;
  const int c = storage_to_node(g, e, &node);
  if (c < 0) return;
  const long long n3 = 3 * g.nn;
  const double d = dinv ? dinv[c * g.nn + node] : 1.0;
  for (int t = 0; t < T; ++t) fields[(long long)t * nstore + e] = d * U[(long long)t * n3 + c * g.nn + node];
}

__global__ void k_ring_field_receivers(GridArgs g, const double* __restrict__ U, int T,
                                       const double* __restrict__ dinv, const int* __restrict__ rx, int n_rx,
                                       int ks, double* d) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= T * n_rx) return;
  const int ch = idx / n_rx, r = idx % n_rx;
  const double* u = U + (long long)ch * 3 * g.nn;
  const int i = rx[2 * r], j = rx[2 * r + 1];
  const double hx = g.h[0][i], hy = g.h[1][j];
  const double inva = -1.0 / (hx * hy);
  const long long e[4] = {0 * g.nn + node_of(g, i, j, ks), 1 * g.nn + node_of(g, i + 1, j, ks),
                          0 * g.nn + node_of(g, i, j + 1, ks), 1 * g.nn + node_of(g, i, j, ks)};
  const double w[4] = {hx * inva, hy * inva, -hx * inva, -hy * inva};
  double acc = 0.0;
  for (int m = 0; m < 4; ++m) acc += w[m] * (dinv ? dinv[e[m]] : 1.0) * u[e[m]];
  d[(long long)ch * n_rx + r] = acc;
}

// out[j][e] = dinv_e * Y_j[node(e)] in storage order (unscaled solutions x_j).
__global__ void k_gather_solutions(GridArgs g, const double2* __restrict__ Y, int J, const double* __restrict__ dinv,
                                   double2* out, long long nstore) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= nstore) return;
  long long node;
  const int c = storage_to_node(g, e, &node);
  if (c < 0) return;
  const double d = dinv[c * g.nn + node];
  for (int j = 0; j < J; ++j) {
    const double2 y = Y[(long long)j * 3 * g.nn + c * g.nn + node];
    out[(long long)j * nstore + e] = make_double2(d * y.x, d * y.y);
  }
}

// padded <- w * storage (entries of padding nodes untouched) and storage <- w * padded.
__global__ void k_scatter_storage(GridArgs g, const double2* __restrict__ xpub, const double* __restrict__ w,
                                  double2* xpad, long long nstore) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= nstore) return;
  long long node;
  const int c = storage_to_node(g, e, &node);
  if (c < 0) return;
  const double s = w[c * g.nn + node];
  const double2 x = xpub[e];
  xpad[c * g.nn + node] = make_double2(s * x.x, s * x.y);
}
__global__ void k_gather_storage(GridArgs g, const double2* __restrict__ xpad, const double* __restrict__ w,
                                 double2* xpub, long long nstore) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= nstore) return;
  long long node;
  const int c = storage_to_node(g, e, &node);
  if (c < 0) return;
  const double s = w[c * g.nn + node];
  const double2 x = xpad[c * g.nn + node];
  xpub[e] = make_double2(s * x.x, s * x.y);
}

// ---------------------------------------------------------------------------
// Adjoint (Sec. 4): batched COCG for the J complex-symmetric systems
//   (A + s_j) mu_j = h_j,   h_j = M^-1/2 g_j,   g_j = sum_k c_jk Q^T w_k,
// then lambda_j = M^-1/2 mu_j and the per-cell gradient.  COCG uses the
// bilinear form x^T y (no conjugation), which is the right inner product for
// the complex symmetric A + s_j.
// ---------------------------------------------------------------------------
// h_j = dinv * sum_r gamma_jr q_r, q_r = -(face circulation)/(face area); one
// thread per shift walks the receivers in order (adjacent faces share edges).
__global__ void k_adj_rhs(GridArgs g, int J, int n_rx, const int* __restrict__ rx, int ks,
                          const double* __restrict__ gamma, const double* __restrict__ dinv, double2* H) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  double2* h = H + (long long)j * 3 * g.nn;
  for (int r = 0; r < n_rx; ++r) {
    const int i = rx[2 * r], jj = rx[2 * r + 1];
    const double hx = g.h[0][i], hy = g.h[1][jj];
    const double inva = -1.0 / (hx * hy);
    const long long e[4] = {0 * g.nn + node_of(g, i, jj, ks), 1 * g.nn + node_of(g, i + 1, jj, ks),
                            0 * g.nn + node_of(g, i, jj + 1, ks), 1 * g.nn + node_of(g, i, jj, ks)};
    const double w[4] = {hx * inva, hy * inva, -hx * inva, -hy * inva};
    const double gr = gamma[2 * ((long long)j * n_rx + r)], gi = gamma[2 * ((long long)j * n_rx + r) + 1];
    for (int m = 0; m < 4; ++m) {
      const double s = w[m] * dinv[e[m]];
      double2 v = h[e[m]];
      v.x += s * gr;
      v.y += s * gi;
      h[e[m]] = v;
    }
  }
}


// init: mu = 0, r = h, p_old = 0; rho = r^T r, |h|^2 (partials per shift)
template <typename V>
__global__ void k_cocg_init(long long n3, int J, const double2* __restrict__ H, V* Mu, V* Rr, V* Pold,
                            double* partials, unsigned int* counter, CocgState* st) {
  __shared__ double red[8];
  __shared__ int flag;
  const int j = blockIdx.y;
  const int nbx = gridDim.x;
  double a_re = 0.0, a_im = 0.0, a_n = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)nbx * blockDim.x) {
    const long long o = (long long)j * n3 + e;
    const cplx hv = as_stored(Rr, ldv(H, o));  // the residual as stored (rounded for FP32 storage)
    stv(Rr, o, hv);
    const double2 h = make_double2(hv.re, hv.im);
    stv(Mu, o, cplx{0.0, 0.0});
    stv(Pold, o, cplx{0.0, 0.0});
    a_re += h.x * h.x - h.y * h.y;
    a_im += 2.0 * h.x * h.y;
    a_n += h.x * h.x + h.y * h.y;
  }
  const double s_re = block_sum(a_re, red), s_im = block_sum(a_im, red), s_n = block_sum(a_n, red);
  const int bid = j * nbx + blockIdx.x;
  if (threadIdx.x == 0) {
    partials[3 * bid] = s_re;
    partials[3 * bid + 1] = s_im;
    partials[3 * bid + 2] = s_n;
  }
  if (!publish_partial(0.0, partials + 3 * gridDim.x * gridDim.y, counter, bid, nbx * gridDim.y, &flag)) return;
  const int t = threadIdx.x;
  if (t < J) {
    double r = 0, i = 0, n = 0;
    for (int b = 0; b < nbx; ++b) {
      const long long q = 3LL * (t * nbx + b);
      r += __hip_atomic_load(partials + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      i += __hip_atomic_load(partials + q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      n += __hip_atomic_load(partials + q + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    st->rho_re[t] = r;
    st->rho_im[t] = i;
    st->hn2[t] = n;
    st->rn2[t] = n;
    st->beta_re[t] = st->beta_im[t] = 0.0;
    st->alpha_re[t] = st->alpha_im[t] = 0.0;
    st->iters[t] = 0;
    st->active[t] = n > 0.0 ? 1 : 0;
  }
  __syncthreads();
  if (t == 0) {
    int na = 0;
    for (int q = 0; q < J; ++q) na += st->active[q];
    st->n_active = na;
    st->breakdown = 0;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// p_j = r_j + beta_j p_j ; q_j = (A + s_j) p_j ; partial p^T q per (shift, block)
template <typename V>
__global__ void __launch_bounds__(CTX* CTY) k_cocg_stencil(GridArgs g, const V* __restrict__ Rr,
                                                           const V* __restrict__ Pold, V* Pnew,
                                                           V* Q, const double* __restrict__ dinv,
                                                           const double* sre, const double* sim, int zblocks,
                                                           double* partials, unsigned int* counter, CocgState* st) {
  __shared__ double red[16];
  __shared__ int flag;
  const int vec = blockIdx.z / zblocks;
  const int zb = blockIdx.z % zblocks;
  const long long off = (long long)vec * 3 * g.nn;
  const bool act = st->active[vec] != 0;
  const cplx beta{st->beta_re[vec], st->beta_im[vec]};
  const double shr = sre[vec], shi = sim[vec];
  double d_re = 0.0, d_im = 0.0;
  if (act) {
    auto load = [&](long long v, int c) {
      const cplx r = ldv(Rr, off + c * g.nn + v), p = ldv(Pold, off + c * g.nn + v);
      return cplx{r.re + beta.re * p.re - beta.im * p.im, r.im + beta.re * p.im + beta.im * p.re};
    };
    auto emit = [&](long long v, int c, cplx kp, cplx u, double d) {
      const long long e = c * g.nn + v;
      cplx out{0.0, 0.0};
      if (d != 0.0) out = cplx{d * kp.re + shr * u.re - shi * u.im, d * kp.im + shr * u.im + shi * u.re};
      stv(Pnew, off + e, u);
      stv(Q, off + e, out);
      d_re += u.re * out.re - u.im * out.im;
      d_im += u.re * out.im + u.im * out.re;
    };
    stencil_tile<cplx, CTX, CTY, CKZ>(g, dinv, zb, load, emit);
  }
  const int nbv = gridDim.x * gridDim.y * zblocks;
  const int bid = vec * nbv + blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * zb);
  const double s_re = block_sum(d_re, red), s_im = block_sum(d_im, red);
  if (flat_tid() == 0) {
    partials[2 * bid] = s_re;
    partials[2 * bid + 1] = s_im;
  }
  const int nb_all = nbv * (gridDim.z / zblocks);
  if (!publish_partial(0.0, partials + 2 * nb_all, counter, bid, nb_all, &flag)) return;
  const int t = flat_tid();
  if (t < st->J && st->active[t]) {
    double r = 0, i = 0;
    for (int b = 0; b < nbv; ++b) {
      const long long q = 2LL * (t * nbv + b);
      r += __hip_atomic_load(partials + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      i += __hip_atomic_load(partials + q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const cplx pq{r, i};
    const cplx al = cdiv(cplx{st->rho_re[t], st->rho_im[t]}, pq);
    if (!(isfinite(al.re) && isfinite(al.im)) || (r == 0.0 && i == 0.0)) {
      st->breakdown = 1;
      st->active[t] = 0;
      st->alpha_re[t] = st->alpha_im[t] = 0.0;
    } else {
      st->alpha_re[t] = al.re;
      st->alpha_im[t] = al.im;
    }
  }
  if (t == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// mu_j += alpha_j p_j ; r_j -= alpha_j q_j ; rho_j' = r^T r ; |r|^2 ; beta_j = rho'/rho
template <typename V>
__global__ void k_cocg_update(long long n3, int J, V* Mu, V* Rr, const V* __restrict__ Pn, const V* __restrict__ Q,
                              double* partials, unsigned int* counter, CocgState* st) {
  __shared__ double red[8];
  __shared__ int flag;
  const int j = blockIdx.y;
  const int nbx = gridDim.x;
  const bool act = st->active[j] != 0;
  const cplx al{st->alpha_re[j], st->alpha_im[j]};
  double a_re = 0.0, a_im = 0.0, a_n = 0.0;
  if (act) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)nbx * blockDim.x) {
      const long long o = (long long)j * n3 + e;
      const cplx p = ldv(Pn, o), q = ldv(Q, o);
      cplx m = ldv(Mu, o), rv = ldv(Rr, o);
      m.re += al.re * p.re - al.im * p.im;
      m.im += al.re * p.im + al.im * p.re;
      rv.re -= al.re * q.re - al.im * q.im;
      rv.im -= al.re * q.im + al.im * q.re;
      stv(Mu, o, m);
      // the dot products see the residual as stored
      const cplx rs = as_stored(Rr, rv);
      stv(Rr, o, rs);
      const double2 r = make_double2(rs.re, rs.im);
      a_re += r.x * r.x - r.y * r.y;
      a_im += 2.0 * r.x * r.y;
      a_n += r.x * r.x + r.y * r.y;
    }
  }
  const double s_re = block_sum(a_re, red), s_im = block_sum(a_im, red), s_n = block_sum(a_n, red);
  const int bid = j * nbx + blockIdx.x;
  if (threadIdx.x == 0) {
    partials[3 * bid] = s_re;
    partials[3 * bid + 1] = s_im;
    partials[3 * bid + 2] = s_n;
  }
  if (!publish_partial(0.0, partials + 3 * gridDim.x * gridDim.y, counter, bid, nbx * gridDim.y, &flag)) return;
  const int t = threadIdx.x;
  if (t < J && st->active[t]) {
    double r = 0, i = 0, n = 0;
    for (int b = 0; b < nbx; ++b) {
      const long long q = 3LL * (t * nbx + b);
      r += __hip_atomic_load(partials + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      i += __hip_atomic_load(partials + q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      n += __hip_atomic_load(partials + q + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const cplx rho_new{r, i}, rho{st->rho_re[t], st->rho_im[t]};
    const cplx be = cdiv(rho_new, rho);
    st->beta_re[t] = be.re;
    st->beta_im[t] = be.im;
    st->rho_re[t] = r;
    st->rho_im[t] = i;
    st->rn2[t] = n;
    st->iters[t] += 1;
    if (!(isfinite(be.re) && isfinite(be.im) && isfinite(n))) {
      st->breakdown = 1;
      st->active[t] = 0;
    } else if (n <= st->tol2 * st->hn2[t] || st->iters[t] >= st->cap[t]) {
      st->active[t] = 0;
    }
  }
  __syncthreads();
  if (t == 0) {
    int na = 0;
    for (int q = 0; q < J; ++q) na += st->active[q];
    st->n_active = na;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Jacobian action (Sec. 4): for a change dm of ln sigma per cell,
//   dM_e = 1/4 sum over the cells around edge e of dm_c sigma_c V_c   (dM/dm . dm),
//   (K + s_j M) dx_j = -s_j dM x_j,
// in the scaled variables (x = D y, dx = D dy, D = M^-1/2):
//   (A + s_j) dy_j = h_j,   h_j[e] = -s_j (dM_e / M_e) y_j[e].
// One thread per padded entry writes h_j for every shift.
__global__ void k_jvp_rhs(GridArgs g, int J, const double* __restrict__ sigma, const double* __restrict__ dm,
                          const double* __restrict__ mass, const double* __restrict__ sre,
                          const double* __restrict__ sim, const double2* __restrict__ Y, double2* H) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= g.nn) return;
  const int i = (int)(v % g.px);
  const int j = (int)((v / g.px) % g.py);
  const int k = (int)(v / ((long long)g.px * g.py));
  auto sv = [&](int ci, int cj, int ck) {
    const long long c = ((long long)ck * g.ny + cj) * g.nx + ci;
    return dm[c] * sigma[c] * g.h[0][ci] * g.h[1][cj] * g.h[2][ck];
  };
  double d[3] = {0.0, 0.0, 0.0};
  if (i < g.nx && j > 0 && j < g.ny && k > 0 && k < g.nz)
    d[0] = 0.25 * (sv(i, j - 1, k - 1) + sv(i, j, k - 1) + sv(i, j - 1, k) + sv(i, j, k));
  if (j < g.ny && i > 0 && i < g.nx && k > 0 && k < g.nz)
    d[1] = 0.25 * (sv(i - 1, j, k - 1) + sv(i, j, k - 1) + sv(i - 1, j, k) + sv(i, j, k));
  if (k < g.nz && i > 0 && i < g.nx && j > 0 && j < g.ny)
    d[2] = 0.25 * (sv(i - 1, j - 1, k) + sv(i, j - 1, k) + sv(i - 1, j, k) + sv(i, j, k));
  const long long n3 = 3 * g.nn;
  for (int c = 0; c < 3; ++c) {
    const long long e = c * g.nn + v;
    const double m = mass[e];
    const double w = m > 0.0 ? d[c] / m : 0.0;
    for (int q = 0; q < J; ++q) {
      const double2 y = Y[(long long)q * n3 + e];
      // -s (w y), s = (sre + i sim)
      const double wr = w * y.x, wi = w * y.y;
      H[(long long)q * n3 + e] = make_double2(-(sre[q] * wr - sim[q] * wi), -(sre[q] * wi + sim[q] * wr));
    }
  }
}

// z_e += sum_j Re(s_j mu_j[e] y_j[e]) / M_e  (lambda_j x_j with lambda = D mu, x = D y)
__global__ void k_grad_edges(long long n3, int J, const double2* __restrict__ Mu, const double2* __restrict__ Y,
                             const double* __restrict__ dinv, const double* sre, const double* sim, double* z) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const double d = dinv[e];
  if (d == 0.0) return;
  double acc = 0.0;
  for (int j = 0; j < J; ++j) {
    const double2 m = Mu[(long long)j * n3 + e], y = Y[(long long)j * n3 + e];
    const double pr = m.x * y.x - m.y * y.y, pi = m.x * y.y + m.y * y.x;
    acc += sre[j] * pr - sim[j] * pi;
  }
  z[e] += acc * d * d;
}

// grad_c = -(sigma_c V_c / 4) sum over the 12 edges of cell c of z_e
__global__ void k_grad_cells(GridArgs g, const double* __restrict__ sigma, const double* __restrict__ z,
                             double* grad) {
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long ncell = (long long)g.nx * g.ny * g.nz;
  if (c >= ncell) return;
  const int i = (int)(c % g.nx), j = (int)((c / g.nx) % g.ny), k = (int)(c / ((long long)g.nx * g.ny));
  double s = 0.0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      s += z[0 * g.nn + node_of(g, i, j + a, k + b)];
      s += z[1 * g.nn + node_of(g, i + a, j, k + b)];
      s += z[2 * g.nn + node_of(g, i + a, j + b, k)];
    }
  const double vol = g.h[0][i] * g.h[1][j] * g.h[2][k];
  grad[c] = -0.25 * sigma[c] * vol * s;
}

// Mu_j += gamma_j Yr_j for all shifts j (complex scalar times complex vector)
__global__ void k_caxpy_shifts(long long n3, int J, const double* __restrict__ gamma, const double2* __restrict__ Yr,
                               double2* Mu) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= n3) return;
  for (int j = 0; j < J; ++j) {
    const double gr = gamma[2 * j], gi = gamma[2 * j + 1];
    const double2 y = Yr[(long long)j * n3 + e];
    double2 m = Mu[(long long)j * n3 + e];
    m.x += gr * y.x - gi * y.y;
    m.y += gr * y.y + gi * y.x;
    Mu[(long long)j * n3 + e] = m;
  }
}

// For J node-padded complex vectors of n3 entries (FP32 storage widened to
// FP64): sign 0 sets Y_j = X_j for every j; sign +1 / -1 adds / subtracts X_j
// for the shifts j whose bit is set in mask.
template <typename V>
__global__ void k_accumulate(long long n3, int J, const V* __restrict__ X, double2* Y, int sign,
                             unsigned long long mask) {
  const long long total = n3 * J;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e / n3);
    if (sign != 0 && !((mask >> j) & 1ull)) continue;
    const cplx x = ldv(X, e);
    if (sign == 0) {
      Y[e] = make_double2(x.re, x.im);
    } else {
      double2 y = Y[e];
      y.x += sign * x.re;
      y.y += sign * x.im;
      Y[e] = y;
    }
  }
}

// Per shift j: (w_j, rho_j) = sum conj(w) rho (re, im) and (w_j, w_j), as
// per-block partials at partials[(3 j + m) * gridDim.x + block].
__global__ void k_dot_shifts(long long n3, const double2* __restrict__ W, const double2* __restrict__ Rh,
                             double* partials) {
  __shared__ double red[8];
  const int j = blockIdx.y;
  double a_re = 0.0, a_im = 0.0, a_n = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)gridDim.x * blockDim.x) {
    const double2 w = W[(long long)j * n3 + e], r = Rh[(long long)j * n3 + e];
    a_re += w.x * r.x + w.y * r.y;
    a_im += w.x * r.y - w.y * r.x;
    a_n += w.x * w.x + w.y * w.y;
  }
  const double s_re = block_sum(a_re, red), s_im = block_sum(a_im, red), s_n = block_sum(a_n, red);
  if (threadIdx.x == 0) {
    const long long nb = gridDim.x;
    partials[(3LL * j + 0) * nb + blockIdx.x] = s_re;
    partials[(3LL * j + 1) * nb + blockIdx.x] = s_im;
    partials[(3LL * j + 2) * nb + blockIdx.x] = s_n;
  }
}

int grid_1d(long long n, int threads, int cap) {
  long long b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace

long long storage_edges(const GridArgs& g) {
  return (long long)g.nx * g.py * g.pz + (long long)g.px * g.ny * g.pz + (long long)g.px * g.py * g.nz;
}


int batch_tiles(const GridArgs& g, int* ntx, int* nty) {
  *ntx = (g.nx + kBTX - 1) / kBTX;
  *nty = (g.ny + kBTY - 1) / kBTY;
  return *ntx * *nty * ((g.nz + kBKZ - 1) / kBKZ);
}

int block_update_blocks(const GridArgs& g) { return grid_1d(3 * g.nn, BU_T, 4096); }

void launch_mass(const GridArgs& g, const double* sigma_cell, double* mass, double* dinv, double* sqrtm,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_mass, dim3((unsigned)((g.nn + 255) / 256)), dim3(256), 0, s, g, sigma_cell, mass, dinv,
                     sqrtm);
}

void launch_scale(long long n, const double* a, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, x, y);
}

void launch_zero2(long long n, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_zero2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, y);
}

void launch_store2(double* p, double a, double b, hipStream_t s) {
  hipLaunchKernelGGL(k_store2, dim3(1), dim3(64), 0, s, p, a, b);
}

void launch_to_complex(long long n, const double* x, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_to_complex, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x, y);
}

template <typename YV, typename PV>
static void seed_init(const GridArgs& g, const double* gvec, double* r0, double* pold, YV* Y, PV* P, int J,
                      Reduce red, SolveState* st, hipStream_t s, const double* r0_scale) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL((k_seed_init<YV, PV>), dim3(UPD_BLOCKS), dim3(UPD_T), 0, s, n3, gvec, r0, pold, Y, P, J,
                     red.partials + kReduceSlots, st, r0_scale);
}
void launch_seed_init(const GridArgs& g, const double* gvec, double* r0, double* pold, double2* Y, double2* P,
                      int J, Reduce red, SolveState* st, hipStream_t s, const double* r0_scale) {
  seed_init(g, gvec, r0, pold, Y, P, J, red, st, s, r0_scale);
}
void launch_seed_init(const GridArgs& g, const double* gvec, double* r0, double* pold, double2* Y, float2* P,
                      int J, Reduce red, SolveState* st, hipStream_t s, const double* r0_scale) {
  seed_init(g, gvec, r0, pold, Y, P, J, red, st, s, r0_scale);
}

// Seed stencil tile shapes (TX x TY node columns, KZ planes per block); the
// variant is chosen per grid (see pick_seed_tile) or by TEM_SEED_TILE.
struct TileShape {
  int tx, ty, kz;
};
static const TileShape kSeedTiles[] = {{32, 4, 2}, {32, 4, 4}, {64, 2, 2}, {64, 2, 4}, {64, 4, 4},
                                       {64, 4, 8}, {32, 8, 4}, {32, 2, 2}, {64, 1, 4}, {64, 2, 8},
                                       {32, 4, 2}, {32, 4, 4}, {64, 2, 2}, {64, 4, 2}, {32, 8, 2}, {64, 2, 4},
                                       {64, 4, 1}, {64, 8, 1}, {32, 8, 1}, {64, 2, 1}, {64, 8, 2}};
constexpr int kNumSeedTiles = (int)(sizeof(kSeedTiles) / sizeof(kSeedTiles[0]));
static int pick_seed_tile(const GridArgs& g) {
  return g.seed_tile >= 0 && g.seed_tile < kNumSeedTiles ? g.seed_tile : 17;
}

static long long seed_tiles_of(const GridArgs& g, const TileShape& t) {
  return (long long)((g.nx + t.tx - 1) / t.tx) * ((g.ny + t.ty - 1) / t.ty) * ((g.nz + t.kz - 1) / t.kz);
}

// (64, 8, 1) tiles, two resident per CU, unless they fill every CU at least
// twice while (64, 8, 2) tiles (one per CU, 107 KB of LDS) fit in a single
// round: then the two-plane tile re-reads a third fewer halo values per node
// and was measured 3.7% faster per launch (64^3); with several rounds the
// one-plane tile is faster (128^3).
int choose_seed_tile(const GridArgs& g, int n_cu) {
  constexpr int kOnePlane = 17, kTwoPlane = 20;
  // TEM_SEED_TILE (an index into the table) overrides the choice for
  // contexts created while it is set
  if (const char* env = getenv("TEM_SEED_TILE")) {
    const int t = atoi(env);
    if (t >= 0 && t < kNumSeedTiles) return t;
  }
  if (n_cu > 0 && seed_tiles_of(g, kSeedTiles[kOnePlane]) >= 2LL * n_cu &&
      seed_tiles_of(g, kSeedTiles[kTwoPlane]) <= n_cu)
    return kTwoPlane;
  return kOnePlane;
}

static dim3 seed_stencil_grid(const GridArgs& g) {
  const TileShape t = kSeedTiles[pick_seed_tile(g)];
  return dim3((g.nx + t.tx - 1) / t.tx, (g.ny + t.ty - 1) / t.ty, (g.nz + t.kz - 1) / t.kz);
}

// Put one kernel into k: a launch on k.stream (with t0 != nullptr the
// dispatch itself records its start and stop events, the kernel's own
// execution interval with no extra packets), or a kernel node of k.graph after
// k.last.  The arguments are converted to the kernel's parameter types first;
// both the launch and the node take copies of them.
template <typename... P, typename... A>
static void put(Sink& k, void (*kernel)(P...), dim3 grid, dim3 block, uint32_t shm, hipEvent_t t0, hipEvent_t t1,
                A... args) {
  static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
  std::tuple<P...> vals(args...);
  void* params[sizeof...(P)];
  std::apply([&](auto&... v) {
    int i = 0;
    ((params[i++] = (void*)&v), ...);
  }, vals);
  void* fn = reinterpret_cast<void*>(kernel);
  if (!k.graph) {
    if (t0) (void)hipExtLaunchKernel(fn, grid, block, params, shm, k.stream, t0, t1, 0);
    else (void)hipLaunchKernel(fn, grid, block, params, shm, k.stream);
    return;
  }
  if (k.err != hipSuccess) return;
  hipKernelNodeParams np{};
  np.func = fn;
  np.gridDim = grid;
  np.blockDim = block;
  np.sharedMemBytes = shm;
  np.kernelParams = params;
  np.extra = nullptr;
  hipGraphNode_t node = nullptr;
  k.err = hipGraphAddKernelNode(&node, k.graph, k.last ? &k.last : nullptr, k.last ? 1 : 0, &np);
  if (k.err == hipSuccess) k.last = node;
}

bool seed_stencil_unscaled_tile(const GridArgs& g) {
  const int v = pick_seed_tile(g);
  return v == 17 || v == 20;
}

void launch_seed_stencil(const GridArgs& g, const double* r, const double* pold, double* pnew, double* q,
                         const double* dinv, double s0, Reduce red, SolveState* st, int local, bool unscaled,
                         Sink& k, hipEvent_t t0, hipEvent_t t1) {
  const int v = pick_seed_tile(g);
  const TileShape t = kSeedTiles[v];
  const dim3 grid = seed_stencil_grid(g), block(t.tx, t.ty);
  const double* up = red.partials + kReduceSlots;
  if (unscaled && v == 17) {
    put(k, k_seed_stencil<64, 8, 1, true, true>, grid, block, 0u, t0, t1, g, r, pold, pnew, q, dinv, s0, up,
        red.partials, st, local);
    return;
  }
  if (unscaled && v == 20) {
    put(k, k_seed_stencil<64, 8, 2, true, true>, grid, block, 0u, t0, t1, g, r, pold, pnew, q, dinv, s0, up,
        red.partials, st, local);
    return;
  }
#define TEM_SEED_CASE(I, X, Y, Z)                                                                            \
  case I:                                                                                                    \
    put(k, k_seed_stencil<X, Y, Z, (I >= 10)>, grid, block, 0u, t0, t1, g, r, pold, pnew, q, dinv, s0, up,      \
        red.partials, st, local);                                                                            \
    break;
  switch (v) {
    TEM_SEED_CASE(0, 32, 4, 2)
    TEM_SEED_CASE(1, 32, 4, 4)
    TEM_SEED_CASE(2, 64, 2, 2)
    TEM_SEED_CASE(3, 64, 2, 4)
    TEM_SEED_CASE(4, 64, 4, 4)
    TEM_SEED_CASE(5, 64, 4, 8)
    TEM_SEED_CASE(6, 32, 8, 4)
    TEM_SEED_CASE(7, 32, 2, 2)
    TEM_SEED_CASE(8, 64, 1, 4)
    TEM_SEED_CASE(9, 64, 2, 8)
    TEM_SEED_CASE(10, 32, 4, 2)
    TEM_SEED_CASE(11, 32, 4, 4)
    TEM_SEED_CASE(12, 64, 2, 2)
    TEM_SEED_CASE(13, 64, 4, 2)
    TEM_SEED_CASE(14, 32, 8, 2)
    TEM_SEED_CASE(15, 64, 2, 4)
    TEM_SEED_CASE(16, 64, 4, 1)
    TEM_SEED_CASE(17, 64, 8, 1)
    TEM_SEED_CASE(18, 32, 8, 1)
    TEM_SEED_CASE(19, 64, 2, 1)
    TEM_SEED_CASE(20, 64, 8, 2)
  }
#undef TEM_SEED_CASE
}

// The one-kernel seed step uses the (64, 8, 2) tile (g.step_kz = 2) or the
// (64, 8, 1) tile.  With three staged vectors the two-plane tile was faster
// at 64^3 and 128^3 alike (15.3 and 126 us against 21.4 and 180 us per step
// in a standalone timing), unlike the two-kernel stencil at 128^3.
static dim3 seed_step_grid(const GridArgs& g, bool* two_plane) {
  *two_plane = g.step_kz != 1;
  const int kz = *two_plane ? 2 : 1;
  return dim3((g.nx + 63) / 64, (g.ny + 7) / 8, (g.nz + kz - 1) / kz);
}

int seed_step_blocks(const GridArgs& g) {
  bool two;
  const dim3 d = seed_step_grid(g, &two);
  return d.x * d.y * d.z;
}

void launch_seed_step(const GridArgs& g, const double* r, const double* p, const double* q, double* rn, double* pn,
                      double* qn, const double* dinv, double s0, Reduce red, SolveState* st, int local, int first,
                      Sink& k, hipEvent_t t0, hipEvent_t t1) {
  bool two;
  const dim3 grid = seed_step_grid(g, &two), block(64, 8);
  const int in = first ? 1 : (local & 1);  // the prologue reads an unused set
  const double* pin = red.partials + (size_t)in * 4 * kReduceSlots;
  double* pout = red.partials + (size_t)(1 - in) * 4 * kReduceSlots;
  if (first) pout = red.partials;  // step 0's partials: set 0
#define TEM_STEP(X, Y, Z, XS) \
  put(k, k_seed_step<X, Y, Z, XS>, grid, block, 0u, t0, t1, g, r, p, q, rn, pn, qn, dinv, s0, pin, pout, st, local, first)
  if (two) TEM_STEP(64, 8, 2, true);
  else TEM_STEP(64, 8, 1, true);
#undef TEM_STEP
}

void launch_shift_block_step(const GridArgs& g, int J, Reduce red, SolveState* st, Sink& k, int f) {
  (void)g;
  put(k, k_shift_block, dim3(J), dim3(64), 0u, nullptr, nullptr, (const double*)red.partials, 0, st, f);
}

void launch_seed_update(const GridArgs& g, const double* r, const double* q, double* rnext, Reduce red,
                        SolveState* st, int local, const double* wd, Sink& k, hipEvent_t t0, hipEvent_t t1) {
  const long long n3 = 3 * g.nn;
  const dim3 sg = seed_stencil_grid(g);
  const int nst = sg.x * sg.y * sg.z;
  put(k, k_seed_update, dim3(UPD_BLOCKS), dim3(UPD_T), 0u, t0, t1, n3, r, q, rnext, (const double*)red.partials, nst,
      red.partials + kReduceSlots, st, local, wd);
}

int seed_stencil_blocks(const GridArgs& g) {
  const dim3 sg = seed_stencil_grid(g);
  return sg.x * sg.y * sg.z;
}

void launch_shift_block(const GridArgs& g, int J, Reduce red, SolveState* st, Sink& k, int f) {
  (void)g;
  put(k, k_shift_block, dim3(J), dim3(64), 0u, nullptr, nullptr, (const double*)(red.partials + kReduceSlots),
      UPD_BLOCKS, st, f);
}

void launch_seed_stencil_batch(const BatchJob* jobs, int njobs, int total_tiles, int B, int local, Sink& k) {
  put(k, k_seed_stencil_batch, dim3(total_tiles), dim3(kBTX, kBTY), 0u, nullptr, nullptr, jobs, njobs, B, local);
}

void launch_seed_update_batch(const BatchJob* jobs, int njobs, int B, int local, Sink& k) {
  put(k, k_seed_update_batch, dim3(UPD_BLOCKS * njobs), dim3(UPD_T), 0u, nullptr, nullptr, jobs, B, local);
}

void launch_shift_block_batch(const BatchJob* jobs, int njobs, int max_J, Sink& k) {
  put(k, k_shift_block_batch, dim3(max_J, njobs), dim3(64), 0u, nullptr, nullptr, jobs);
}

void launch_block_update_batch(const BatchJob* jobs, int njobs, int total_blocks, int B, Sink& k) {
  const dim3 grid(total_blocks), block(BU_T);
  switch (B) {
    case 16: put(k, k_block_update_batch<16>, grid, block, 0u, nullptr, nullptr, jobs, njobs); break;
    case 32: put(k, k_block_update_batch<32>, grid, block, 0u, nullptr, nullptr, jobs, njobs); break;
    case 64: put(k, k_block_update_batch<64>, grid, block, 0u, nullptr, nullptr, jobs, njobs); break;
    default: put(k, k_block_update_batch<8>, grid, block, 0u, nullptr, nullptr, jobs, njobs); break;
  }
}

void launch_gather_heads(const BatchJob* jobs, int njobs, SolveHead* out, Sink& k) {
  put(k, k_gather_heads, dim3(njobs), dim3(64), 0u, nullptr, nullptr, jobs, njobs, out);
}


template <typename YV, typename PV>
static void block_update(const GridArgs& g, const double* R, const double* R0, YV* Y, PV* P, int J, int B,
                         const SolveState* st, Sink& k, int f, int max_blocks, const double* rs) {
  const long long n3 = 3 * g.nn;
  const dim3 grid(grid_1d(n3, BU_T, max_blocks)), block(BU_T);
  switch (B) {
    case 16: put(k, k_block_update<16, YV, PV>, grid, block, 0u, nullptr, nullptr, n3, R, R0, Y, P, J, st, f, rs); break;
    case 32: put(k, k_block_update<32, YV, PV>, grid, block, 0u, nullptr, nullptr, n3, R, R0, Y, P, J, st, f, rs); break;
    case 64: put(k, k_block_update<64, YV, PV>, grid, block, 0u, nullptr, nullptr, n3, R, R0, Y, P, J, st, f, rs); break;
    default: put(k, k_block_update<8, YV, PV>, grid, block, 0u, nullptr, nullptr, n3, R, R0, Y, P, J, st, f, rs); break;
  }
}
void launch_block_update(const GridArgs& g, const double* R, const double* R0, double2* Y, double2* P, int J, int B,
                         const SolveState* st, Sink& k, int f, int max_blocks, const double* rscale) {
  block_update(g, R, R0, Y, P, J, B, st, k, f, max_blocks, rscale);
}
void launch_block_update(const GridArgs& g, const double* R, const double* R0, double2* Y, float2* P, int J, int B,
                         const SolveState* st, Sink& k, int f, int max_blocks, const double* rscale) {
  block_update(g, R, R0, Y, P, J, B, st, k, f, max_blocks, rscale);
}

void launch_accumulate(const GridArgs& g, int J, const float2* X, double2* Y, int sign, unsigned long long mask,
                       hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_accumulate<float2>, dim3(grid_1d(n3 * J, 256, 8192)), dim3(256), 0, s, n3, J, X, Y, sign,
                     mask);
}

int cstencil_blocks(const GridArgs& g) {
  return ((g.nx + CTX - 1) / CTX) * ((g.ny + CTY - 1) / CTY) * ((g.nz + CKZ - 1) / CKZ);
}

void launch_cstencil(const GridArgs& g, const double2* X, long long xstride, const double* dinv,
                     const double* shift_re, const double* shift_im, int nvec, const double2* rhs, double2* out,
                     long long ostride, double* norm_partials, hipStream_t s) {
  const int zb = (g.nz + CKZ - 1) / CKZ;
  dim3 grid((g.nx + CTX - 1) / CTX, (g.ny + CTY - 1) / CTY, zb * nvec);
  hipLaunchKernelGGL(k_cstencil, grid, dim3(CTX, CTY), 0, s, g, X, xstride, dinv, shift_re, shift_im, rhs, out,
                     ostride, norm_partials, zb);
}

void launch_reduce_rows(const double* partials, int rows, int cols, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(256), 0, s, partials, cols, out);
}

void launch_contract(const GridArgs& g, const double2* Y, int J, const double* dinv, const double* C, int T,
                     double* U, hipStream_t s) {
  const long long ns = storage_edges(g);
  const long long blocks = (ns + 63) / 64;
  hipLaunchKernelGGL(k_contract, dim3((unsigned)blocks), dim3(256), 0, s, g, Y, J, dinv, C, T, U, ns);
}

void launch_receivers(const GridArgs& g, const double2* Y, int J, const double* dinv, const double* C, int T,
                      const int* rx, int n_rx, int k_s, double* d, hipStream_t s) {
  const int n = T * n_rx;
  hipLaunchKernelGGL(k_receivers, dim3((n + 127) / 128), dim3(128), 0, s, g, Y, J, dinv, C, T, rx, n_rx, k_s, d);
}

void launch_ring_receivers(const GridArgs& g, const double* R, int B, const double* dinv, const int* rx, int n_rx,
                           int ks, double* hq, int init, Sink& k) {
  const int n = (init ? 1 : B) * n_rx;
  put(k, k_ring_receivers, dim3((unsigned)((n + 255) / 256)), dim3(256), 0u, nullptr, nullptr, g, R, B, dinv, rx,
      n_rx, ks, hq, init);
}

void launch_ring_contract_init(const GridArgs& g, const double* r0, const double* W, int T, double* U, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_ring_contract_init, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3, r0, W, T, U);
}

void launch_ring_contract(const GridArgs& g, const double* R, int B, const double* W, int T, double* U,
                          const SolveState* st, Sink& k) {
  const long long n3 = 3 * g.nn;
  const unsigned blocks = (unsigned)((n3 + 63) / 64);
  put(k, k_ring_contract, dim3(blocks), dim3(256), 0u, nullptr, nullptr, n3, R, B, W, T, U, st);
}

void launch_ring_fields(const GridArgs& g, const double* U, int T, const double* dinv, double* fields,
                        const int* rx, int n_rx, int ks, double* d, hipStream_t s) {
  const long long ns = storage_edges(g);
  if (fields)
    hipLaunchKernelGGL(k_ring_fields, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, g, U, T, dinv, fields, ns);
  if (n_rx > 0)
    hipLaunchKernelGGL(k_ring_field_receivers, dim3((unsigned)((T * n_rx + 255) / 256)), dim3(256), 0, s, g, U, T,
                       dinv, rx, n_rx, ks, d);
}

void launch_gather_solutions(const GridArgs& g, const double2* Y, int J, const double* dinv, double2* out,
                             hipStream_t s) {
  const long long ns = storage_edges(g);
  hipLaunchKernelGGL(k_gather_solutions, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, g, Y, J, dinv, out,
                     ns);
}

void launch_scatter_storage(const GridArgs& g, const double2* xpub, const double* w, double2* xpad, hipStream_t s) {
  const long long ns = storage_edges(g);
  hipLaunchKernelGGL(k_scatter_storage, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, g, xpub, w, xpad, ns);
}

void launch_gather_storage(const GridArgs& g, const double2* xpad, const double* w, double2* xpub, hipStream_t s) {
  const long long ns = storage_edges(g);
  hipLaunchKernelGGL(k_gather_storage, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, g, xpad, w, xpub, ns);
}

int cstencil_partials(const GridArgs& g) { return cstencil_blocks(g); }

size_t cocg_state_bytes() { return sizeof(CocgState); }

int cocg_partials(const GridArgs& g, int J) {
  // row kernels: 3 sums per (shift, block) + one publish slot per block, <= 128 blocks per shift;
  // stencil: 2 sums per block + one publish slot per block, nbv blocks per shift
  const int zb = (g.nz + CKZ - 1) / CKZ;
  const int nbv = ((g.nx + CTX - 1) / CTX) * ((g.ny + CTY - 1) / CTY) * zb;
  return std::max(4 * 128 * J, 3 * nbv * J) + 64;
}

void launch_adj_rhs(const GridArgs& g, int J, int n_rx, const int* rx, int ks, const double* gamma, const double* dinv,
                    double2* H, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_rhs, dim3(1), dim3(64), 0, s, g, J, n_rx, rx, ks, gamma, dinv, H);
}

static int cocg_row_blocks(long long n3) { return grid_1d(n3, 256, 128); }

template <typename V>
static void cocg_init(const GridArgs& g, int J, const double2* H, V* Mu, V* Rr, V* Pold, double* partials,
                      unsigned int* counter, void* st, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_cocg_init<V>, dim3(cocg_row_blocks(n3), J), dim3(256), 0, s, n3, J, H, Mu, Rr, Pold, partials,
                     counter, (CocgState*)st);
}
void launch_cocg_init(const GridArgs& g, int J, const double2* H, double2* Mu, double2* Rr, double2* Pold,
                      double* partials, unsigned int* counter, void* st, hipStream_t s) {
  cocg_init(g, J, H, Mu, Rr, Pold, partials, counter, st, s);
}
void launch_cocg_init(const GridArgs& g, int J, const double2* H, float2* Mu, float2* Rr, float2* Pold,
                      double* partials, unsigned int* counter, void* st, hipStream_t s) {
  cocg_init(g, J, H, Mu, Rr, Pold, partials, counter, st, s);
}

template <typename V>
static void cocg_stencil(const GridArgs& g, int J, const V* Rr, const V* Pold, V* Pnew, V* Q, const double* dinv,
                         const double* sre, const double* sim, double* partials, unsigned int* counter, void* st,
                         hipStream_t s) {
  const int zb = (g.nz + CKZ - 1) / CKZ;
  dim3 grid((g.nx + CTX - 1) / CTX, (g.ny + CTY - 1) / CTY, zb * J);
  hipLaunchKernelGGL(k_cocg_stencil<V>, grid, dim3(CTX, CTY), 0, s, g, Rr, Pold, Pnew, Q, dinv, sre, sim, zb,
                     partials, counter, (CocgState*)st);
}
void launch_cocg_stencil(const GridArgs& g, int J, const double2* Rr, const double2* Pold, double2* Pnew, double2* Q,
                         const double* dinv, const double* sre, const double* sim, double* partials,
                         unsigned int* counter, void* st, hipStream_t s) {
  cocg_stencil(g, J, Rr, Pold, Pnew, Q, dinv, sre, sim, partials, counter, st, s);
}
void launch_cocg_stencil(const GridArgs& g, int J, const float2* Rr, const float2* Pold, float2* Pnew, float2* Q,
                         const double* dinv, const double* sre, const double* sim, double* partials,
                         unsigned int* counter, void* st, hipStream_t s) {
  cocg_stencil(g, J, Rr, Pold, Pnew, Q, dinv, sre, sim, partials, counter, st, s);
}

template <typename V>
static void cocg_update(const GridArgs& g, int J, V* Mu, V* Rr, const V* Pn, const V* Q, double* partials,
                        unsigned int* counter, void* st, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_cocg_update<V>, dim3(cocg_row_blocks(n3), J), dim3(256), 0, s, n3, J, Mu, Rr, Pn, Q, partials,
                     counter, (CocgState*)st);
}
void launch_cocg_update(const GridArgs& g, int J, double2* Mu, double2* Rr, const double2* Pn, const double2* Q,
                        double* partials, unsigned int* counter, void* st, hipStream_t s) {
  cocg_update(g, J, Mu, Rr, Pn, Q, partials, counter, st, s);
}
void launch_cocg_update(const GridArgs& g, int J, float2* Mu, float2* Rr, const float2* Pn, const float2* Q,
                        double* partials, unsigned int* counter, void* st, hipStream_t s) {
  cocg_update(g, J, Mu, Rr, Pn, Q, partials, counter, st, s);
}

void launch_grad_edges(const GridArgs& g, int J, const double2* Mu, const double2* Y, const double* dinv,
                       const double* sre, const double* sim, double* z, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_grad_edges, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3, J, Mu, Y, dinv, sre, sim,
                     z);
}

void launch_caxpy_shifts(const GridArgs& g, int J, const double* gamma, const double2* Yr, double2* Mu,
                         hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_caxpy_shifts, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3, J, gamma, Yr, Mu);
}

int dot_shifts_blocks(const GridArgs& g) { return grid_1d(3 * g.nn, 256, 128); }

void launch_dot_shifts(const GridArgs& g, int J, const double2* W, const double2* Rh, double* partials, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_dot_shifts, dim3(dot_shifts_blocks(g), J), dim3(256), 0, s, n3, W, Rh, partials);
}

void launch_jvp_rhs(const GridArgs& g, int J, const double* sigma, const double* dm, const double* mass,
                    const double* sre, const double* sim, const double2* Y, double2* H, hipStream_t s) {
  hipLaunchKernelGGL(k_jvp_rhs, dim3((unsigned)((g.nn + 255) / 256)), dim3(256), 0, s, g, J, sigma, dm, mass, sre, sim,
                     Y, H);
}

void launch_grad_cells(const GridArgs& g, const double* sigma, const double* z, double* grad, hipStream_t s) {
  const long long nc = (long long)g.nx * g.ny * g.nz;
  hipLaunchKernelGGL(k_grad_cells, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, g, sigma, z, grad);
}


}  // namespace tem
