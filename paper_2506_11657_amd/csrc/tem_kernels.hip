// Device kernels for the shared-pole TEM forward path on gfx950 (CDNA4).
//
// Every operator here acts on the node-padded edge layout described in
// tem_internal.h.  The shifted systems (K + s_j M) x_j = f of eq. (rmj) are
// solved in the symmetric scaling y = M^{1/2} x:
//     (A + s_j) y_j = g,   A = M^{-1/2} K M^{-1/2},   g = M^{-1/2} f,
// where K = C^T W C is applied matrix-free: face circulations of the scaled
// field weighted by h_dual / (mu0 * area), then gathered back onto the edges.
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
__device__ __forceinline__ double zero_of(double) { return 0.0; }
__device__ __forceinline__ cplx zero_of(cplx) { return {0.0, 0.0}; }

__device__ __forceinline__ int flat_tid() { return threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z); }
__device__ __forceinline__ int flat_threads() { return blockDim.x * blockDim.y * blockDim.z; }

// Deterministic block sum (wave64 shuffles, then the waves in fixed order);
// the result is valid in thread 0.  lds needs one double per wave.
__device__ double block_sum(double v, double* lds) {
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_down(v, off, kWave);
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

// Fixed-order sum of n partials by one block.
__device__ double sum_partials(const double* partials, int n, double* lds) {
  double s = 0.0;
  for (int i = flat_tid(); i < n; i += flat_threads())
    s += __hip_atomic_load(partials + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return block_sum(s, lds);
}

__device__ __forceinline__ long long node_of(const GridArgs& g, int i, int j, int k) {
  return ((long long)k * g.py + j) * g.px + i;
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
  __shared__ Val sp[2][3][TY + 2][TX + 2];  // scaled field, two planes
  __shared__ Val phi[3][TY + 1][TX + 1];    // face fluxes of the current plane

  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = tx + TX * ty;
  constexpr int NT = TX * TY;
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;
  const int k0 = zb * KZ;
  const int kend = min(k0 + KZ, g.nz);
  const int i = i0 + tx, j = j0 + ty;
  const bool own = (i < g.nx) && (j < g.ny);

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
        sp[slot][c][lj][li] = (d != 0.0) ? d * load(v, c) : zero_of(Val{});
      }
    }
  };
  // fluxes of the three faces owned by node (gi, gj, kk) whose halo
  // coordinates are (li, lj); zero outside the grid
  auto fluxes = [&](int gi, int gj, int kk, int li, int lj, Val& fx, Val& fy, Val& fz) {
    fx = fy = fz = zero_of(Val{});
    if (gi < 0 || gj < 0 || kk < 0 || gi > g.nx || gj > g.ny || kk > g.nz) return;
    const int s0 = kk & 1, s1 = (kk + 1) & 1;
    const double hxi = g.h[0][gi], hyj = g.h[1][gj], hzk = g.h[2][kk];
    const double wx = g.dw[0][gi] * g.ih[1][gj] * g.ih[2][kk];
    const double wy = g.dw[1][gj] * g.ih[2][kk] * g.ih[0][gi];
    const double wz = g.dw[2][kk] * g.ih[0][gi] * g.ih[1][gj];
    // Fx: +y, +z, -y, -z ; Fy: +z, +x, -z, -x ; Fz: +x, +y, -x, -y
    fx = wx * (hyj * sp[s0][1][lj][li] + hzk * sp[s0][2][lj + 1][li] - hyj * sp[s1][1][lj][li] - hzk * sp[s0][2][lj][li]);
    fy = wy * (hzk * sp[s0][2][lj][li] + hxi * sp[s1][0][lj][li] - hzk * sp[s0][2][lj][li + 1] - hxi * sp[s0][0][lj][li]);
    fz = wz * (hxi * sp[s0][0][lj][li] + hyj * sp[s0][1][lj][li + 1] - hxi * sp[s0][0][lj + 1][li] - hyj * sp[s0][1][lj][li]);
  };

  Val fx_prev = zero_of(Val{}), fy_prev = zero_of(Val{});
  load_plane(k0 - 1);
  load_plane(k0);
  __syncthreads();
  {
    Val fz_unused;
    fluxes(i, j, k0 - 1, tx + 1, ty + 1, fx_prev, fy_prev, fz_unused);
  }
  __syncthreads();

  for (int kk = k0; kk < kend; ++kk) {
    load_plane(kk + 1);  // overwrites plane kk-1, no longer needed
    __syncthreads();
    for (int e = tid; e < (TX + 1) * (TY + 1); e += NT) {
      const int li = e % (TX + 1), lj = e / (TX + 1);
      Val a, b, c;
      fluxes(i0 - 1 + li, j0 - 1 + lj, kk, li, lj, a, b, c);
      phi[0][lj][li] = a;
      phi[1][lj][li] = b;
      phi[2][lj][li] = c;
    }
    __syncthreads();
    if (own) {
      const int li = tx + 1, lj = ty + 1;
      const Val fx = phi[0][lj][li], fy = phi[1][lj][li], fz = phi[2][lj][li];
      // (K p)_Ex = hx (phi_y(k-1) - phi_y + phi_z - phi_z(j-1)), and cyclically
      const Val kpx = g.h[0][i] * (fy_prev - fy + fz - phi[2][lj - 1][li]);
      const Val kpy = g.h[1][j] * (phi[2][lj][li - 1] - fz + fx - fx_prev);
      const Val kpz = g.h[2][kk] * (phi[0][lj - 1][li] - fx + fy - phi[1][lj][li - 1]);
      const long long v = node_of(g, i, j, kk);
      emit(v, 0, kpx);
      emit(v, 1, kpy);
      emit(v, 2, kpz);
      fx_prev = fx;
      fy_prev = fy;
    }
    __syncthreads();
  }
}

constexpr int STX = 32, STY = 8, SKZ = 4;

// ---------------------------------------------------------------------------
// Seed CG, iteration k:
//   stencil: p_k = r_k + beta_{k-1} p_{k-1};  q = A0 p_k = dinv K (dinv p_k) + s0 p_k;
//            alpha_k = (r_k, r_k) / (p_k, q)
//   update:  r_{k+1} = r_k - alpha_k q;  beta_k = (r_{k+1}, r_{k+1}) / (r_k, r_k);
//            shifted recurrences and deferred-update coefficients for every shift.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(STX* STY) k_seed_stencil(GridArgs g, const double* __restrict__ r,
                                                          const double* __restrict__ pold,
                                                          double* __restrict__ pnew, double* __restrict__ q,
                                                          const double* __restrict__ dinv, double s0,
                                                          double* partials, unsigned int* counter,
                                                          SolveState* st) {
  __shared__ double red[16];
  __shared__ int flag;
  const double beta = st->beta;
  double dot = 0.0;
  auto load = [&](long long v, int c) { return r[c * g.nn + v] + beta * pold[c * g.nn + v]; };
  auto emit = [&](long long v, int c, double kp) {
    const long long e = c * g.nn + v;
    const double u = r[e] + beta * pold[e];
    const double d = dinv[e];
    const double out = d * kp + s0 * u;
    pnew[e] = u;
    q[e] = out;
    dot += u * out;
  };
  stencil_tile<double, STX, STY, SKZ>(g, dinv, blockIdx.z, load, emit);
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const double s = block_sum(dot, red);
  if (publish_partial(s, partials, counter, bid, nb, &flag)) {
    const double pap = sum_partials(partials, nb, red);
    if (flat_tid() == 0) {
      st->pAp = pap;
      if (!(pap > 0.0) || !isfinite(pap)) {
        st->breakdown = 1;
        st->alpha = 0.0;
      } else {
        st->alpha = st->rr / pap;
      }
      __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

constexpr int UPD_T = 256;

__global__ void __launch_bounds__(UPD_T) k_seed_update(long long n, const double* __restrict__ r,
                                                       const double* __restrict__ q, double* __restrict__ rnext,
                                                       double* partials, unsigned int* counter, SolveState* st,
                                                       int slot_next) {
  __shared__ double red[8];
  __shared__ int flag;
  __shared__ double sh[2];
  const double alpha = st->alpha;
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)UPD_T + threadIdx.x; e < n; e += (long long)gridDim.x * UPD_T) {
    const double v = r[e] - alpha * q[e];
    rnext[e] = v;
    acc += v * v;
  }
  const double s = block_sum(acc, red);
  if (!publish_partial(s, partials, counter, blockIdx.x, gridDim.x, &flag)) return;
  double rr_next = sum_partials(partials, gridDim.x, red);
  const int t = threadIdx.x;
  if (t == 0) {
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh[0] = rr_next;
    sh[1] = st->rr;
    if (!isfinite(rr_next)) st->breakdown = 1;
  }
  __syncthreads();
  rr_next = sh[0];
  const double rr = sh[1];
  const double beta = rr > 0.0 ? rr_next / rr : 0.0;  // beta_k
  const double a_k = st->alpha, a_km1 = st->alpha_prev, b_km1 = st->beta;
  const int B = st->B;
  const int k = st->k;
  const int local = k % B;
  const int J = st->J;
  int my_active = 0;
  if (t < J) {
    if (local == 0) {  // this step opens a new block of deferred updates
      st->a_re[t] = 1.0;
      st->a_im[t] = 0.0;
      st->c_re[t] = st->c_im[t] = 0.0;
      for (int l = 0; l < B; ++l) st->d_re[t][l] = st->d_im[t][l] = st->e_re[t][l] = st->e_im[t][l] = 0.0;
      st->apply[t] = st->active[t];
    }
    if (st->active[t]) {
      const cplx z{st->z_re[t], st->z_im[t]}, zp{st->zp_re[t], st->zp_im[t]};
      const cplx sig{st->sig_re[t], st->sig_im[t]};
      // zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1} /
      //             (a_k b_{k-1} (zeta_{k-1} - zeta_k) + zeta_{k-1} a_{k-1} (1 + sig a_k))
      const cplx num = a_km1 * cmul(z, zp);
      const cplx one_sa{1.0 + sig.re * a_k, sig.im * a_k};
      const cplx den = (a_k * b_km1) * (zp - z) + a_km1 * cmul(zp, one_sa);
      const cplx zn = cdiv(num, den);
      const cplx ratio = cdiv(zn, z);
      const cplx as = a_k * ratio;                // alpha_k^sigma
      const cplx bs = beta * cmul(ratio, ratio);  // beta_k^sigma
      const bool ok = isfinite(zn.re) && isfinite(zn.im) && isfinite(as.re) && isfinite(as.im) &&
                      isfinite(bs.re) && isfinite(bs.im);
      if (!ok) {
        st->breakdown = 1;
      } else {
        // y_{k+1} = y_k + as p_k  with  p_k = a P + sum_l e_l r_l
        const cplx a{st->a_re[t], st->a_im[t]};
        const cplx c = cplx{st->c_re[t], st->c_im[t]} + cmul(as, a);
        st->c_re[t] = c.re;
        st->c_im[t] = c.im;
        for (int l = 0; l < B; ++l) {
          const cplx e{st->e_re[t][l], st->e_im[t][l]};
          const cplx d = cplx{st->d_re[t][l], st->d_im[t][l]} + cmul(as, e);
          st->d_re[t][l] = d.re;
          st->d_im[t][l] = d.im;
          const cplx en = cmul(bs, e);
          st->e_re[t][l] = en.re;
          st->e_im[t][l] = en.im;
        }
        // p_{k+1} = zeta_{k+1} r_{k+1} + bs p_k
        const cplx an = cmul(bs, a);
        st->a_re[t] = an.re;
        st->a_im[t] = an.im;
        st->e_re[t][slot_next] = zn.re;
        st->e_im[t][slot_next] = zn.im;
        st->zp_re[t] = z.re;
        st->zp_im[t] = z.im;
        st->z_re[t] = zn.re;
        st->z_im[t] = zn.im;
        st->iters[t] += 1;
        const double est2 = (zn.re * zn.re + zn.im * zn.im) * rr_next;
        st->est[t] = sqrt(est2);
        if (est2 <= st->tol2) st->active[t] = 0;
      }
    }
    my_active = st->active[t];
  }
  const double na = block_sum((double)my_active, red);
  if (t == 0) {
    st->n_active = (int)na;
    st->alpha_prev = a_k;
    st->beta = beta;
    st->rr = rr_next;
    st->k = k + 1;
  }
}

// Deferred shift update after a block of BB seed iterations:
//   p_j <- a_j p_j + sum_l e_jl r_l,   y_j <- y_j + c_j p_j + sum_l d_jl r_l
// for every shift updated in the block (coefficients from k_seed_update).
// Coefficients sit in shared memory, (a, c, e_0.., d_0..) per shift.
constexpr int BU_T = 256;
template <int BB>
__global__ void __launch_bounds__(BU_T) k_block_update(long long n3, const double* __restrict__ R, double2* Y,
                                                       double2* P, int J, const SolveState* st) {
  extern __shared__ double cf[];
  __shared__ int app[kMaxShifts];
  constexpr int W = 2 * BB + 2;
  for (int idx = threadIdx.x; idx < J * W; idx += BU_T) {
    const int j = idx / W, m = idx % W;
    double re, im;
    if (m == 0) { re = st->a_re[j]; im = st->a_im[j]; }
    else if (m == 1) { re = st->c_re[j]; im = st->c_im[j]; }
    else if (m < 2 + BB) { re = st->e_re[j][m - 2]; im = st->e_im[j][m - 2]; }
    else { re = st->d_re[j][m - 2 - BB]; im = st->d_im[j][m - 2 - BB]; }
    cf[2 * idx] = re;
    cf[2 * idx + 1] = im;
  }
  for (int j = threadIdx.x; j < J; j += BU_T) app[j] = st->apply[j];
  __syncthreads();
  for (long long e = blockIdx.x * (long long)BU_T + threadIdx.x; e < n3; e += (long long)gridDim.x * BU_T) {
    double rl[BB];
#pragma unroll
    for (int l = 0; l < BB; ++l) rl[l] = R[(long long)l * n3 + e];
    for (int j = 0; j < J; ++j) {
      if (!app[j]) continue;
      const double* c = cf + 2 * j * W;
      const double2 p = P[(long long)j * n3 + e];
      const double2 y = Y[(long long)j * n3 + e];
      double pr = c[0] * p.x - c[1] * p.y;
      double pi = c[0] * p.y + c[1] * p.x;
      double yr = y.x + c[2] * p.x - c[3] * p.y;
      double yi = y.y + c[2] * p.y + c[3] * p.x;
#pragma unroll
      for (int l = 0; l < BB; ++l) {
        pr += c[4 + 2 * l] * rl[l];
        pi += c[5 + 2 * l] * rl[l];
        yr += c[4 + 2 * BB + 2 * l] * rl[l];
        yi += c[5 + 2 * BB + 2 * l] * rl[l];
      }
      P[(long long)j * n3 + e] = make_double2(pr, pi);
      Y[(long long)j * n3 + e] = make_double2(yr, yi);
    }
  }
}

__global__ void k_seed_init(long long n3, const double* __restrict__ gv, double* r0, double* pold, double2* Y,
                            double2* P, int J, double* partials, unsigned int* counter, SolveState* st) {
  __shared__ double red[8];
  __shared__ int flag;
  double acc = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)gridDim.x * blockDim.x) {
    const double v = gv[e];
    r0[e] = v;
    pold[e] = 0.0;
    for (int j = 0; j < J; ++j) {
      Y[(long long)j * n3 + e] = make_double2(0.0, 0.0);
      P[(long long)j * n3 + e] = make_double2(v, 0.0);
    }
    acc += v * v;
  }
  const double s = block_sum(acc, red);
  if (!publish_partial(s, partials, counter, blockIdx.x, gridDim.x, &flag)) return;
  const double rr = sum_partials(partials, gridDim.x, red);
  if (threadIdx.x == 0) {
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st->rr = rr;
    st->rr0 = rr;
    st->tol2 *= rr;  // the host stores rtol^2 here
    st->alpha = 0.0;
    st->beta = 0.0;
    st->alpha_prev = 1.0;
    st->beta_prev = 0.0;
    st->k = 0;
    st->breakdown = (rr > 0.0 && isfinite(rr)) ? 0 : 1;
    st->n_active = st->J;
  }
}

// ---------------------------------------------------------------------------
// Complex shifted operator on nvec vectors, vector index = blockIdx.z / zblocks:
//   out_j = rhs - (A + s_j) X_j   (rhs != nullptr)   or   out_j = (A + s_j) X_j,
// plus per-block partial sums of |out_j|^2 in norm_partials[j * nblocks + b].
// ---------------------------------------------------------------------------
constexpr int CTX = 32, CTY = 4, CKZ = 4;
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
  auto emit = [&](long long v, int c, cplx kp) {
    const long long e = c * g.nn + v;
    const double d = dinv[e];
    cplx res{0.0, 0.0};
    if (d != 0.0) {
      const double2 u = x[e];
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

__global__ void k_to_complex(long long n, const double* x, double2* y) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e < n) y[e] = make_double2(x[e], 0.0);
}

// ---------------------------------------------------------------------------
// Residue contraction (Sec. 3.2, the product S R): fields in storage order,
//   U[k][e] = dinv_e * sum_j Re(C_jk Y_j[e]) = [Re Y | Im Y] [Re C ; -Im C],
// as an (edges x 2J) x (2J x T) product on FP64 MFMA (v_mfma_f64_16x16x4f64).
// One wave computes 16 edges x all channels (T <= 64).
// Lane layout of the 16x16x4 FP64 MFMA: lane l supplies A[l%16][l/16] and
// B[l/16][l%16] and holds D[4*(l/16)+r][l%16], r = 0..3.
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
      const long long e = e0 + 4 * kq + r;
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

int reduce_blocks(long long n) { return grid_1d(n, UPD_T, 1024); }

void launch_mass(const GridArgs& g, const double* sigma_cell, double* mass, double* dinv, double* sqrtm,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_mass, dim3((unsigned)((g.nn + 255) / 256)), dim3(256), 0, s, g, sigma_cell, mass, dinv,
                     sqrtm);
}

void launch_scale(long long n, const double* a, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a, x, y);
}

void launch_to_complex(long long n, const double* x, double2* y, hipStream_t s) {
  hipLaunchKernelGGL(k_to_complex, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, x, y);
}

void launch_seed_init(const GridArgs& g, const double* gvec, double* r0, double* pold, double2* Y, double2* P,
                      int J, Reduce red, SolveState* st, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_seed_init, dim3(reduce_blocks(n3)), dim3(UPD_T), 0, s, n3, gvec, r0, pold, Y, P, J,
                     red.partials, red.counter, st);
}

void launch_seed_stencil(const GridArgs& g, const double* r, const double* pold, double* pnew, double* q,
                         const double* dinv, double s0, Reduce red, SolveState* st, hipStream_t s) {
  dim3 grid((g.nx + STX - 1) / STX, (g.ny + STY - 1) / STY, (g.nz + SKZ - 1) / SKZ);
  hipLaunchKernelGGL(k_seed_stencil, grid, dim3(STX, STY), 0, s, g, r, pold, pnew, q, dinv, s0, red.partials,
                     red.counter, st);
}

void launch_seed_update(const GridArgs& g, const double* r, const double* q, double* rnext, Reduce red,
                        SolveState* st, int slot_next, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  hipLaunchKernelGGL(k_seed_update, dim3(reduce_blocks(n3)), dim3(UPD_T), 0, s, n3, r, q, rnext,
                     red.partials + kReduceSlots, red.counter + 1, st, slot_next);
}

void launch_block_update(const GridArgs& g, const double* R, double2* Y, double2* P, int J, int B,
                         const SolveState* st, hipStream_t s) {
  const long long n3 = 3 * g.nn;
  const dim3 grid(grid_1d(n3, BU_T, 4096)), block(BU_T);
  const size_t shm = (size_t)J * (2 * B + 2) * 2 * sizeof(double);
  switch (B) {
    case 16: hipLaunchKernelGGL(k_block_update<16>, grid, block, shm, s, n3, R, Y, P, J, st); break;
    case 32: hipLaunchKernelGGL(k_block_update<32>, grid, block, shm, s, n3, R, Y, P, J, st); break;
    case 64: hipLaunchKernelGGL(k_block_update<64>, grid, block, shm, s, n3, R, Y, P, J, st); break;
    default: hipLaunchKernelGGL(k_block_update<8>, grid, block, shm, s, n3, R, Y, P, J, st); break;
  }
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

}  // namespace tem
