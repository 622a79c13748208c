// Internal declarations shared by the host orchestration (tem_host.hip),
// the device kernels (tem_kernels.hip) and the host RKFIT (tem_rkfit.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace tem {

constexpr double kMu0 = 4e-7 * 3.14159265358979323846;  // Sec. 2.1
constexpr int kMaxShifts = 64;
constexpr int kMaxBlock = 64;       // deferred-update block length (iterations)
constexpr int kReduceSlots = 4096;  // per-kernel partial sums (upper bound on blocks)

// Node-padded layout: every node (i, j, k), 0 <= i <= nx, ... owns the three
// edges Ex(i,j,k), Ey(i,j,k), Ez(i,j,k) leaving it in +x, +y, +z.  Edges that
// do not exist (Ex at i = nx, ...) and PEC boundary edges are kept as zeros.
// A real field is 3 * nn doubles: component c of node v at c * nn + v, with
// v = (k * py + j) * px + i, px = nx + 1, py = ny + 1.
struct GridArgs {
  int nx, ny, nz;
  int px, py, pz;
  long long nn;             // px * py * pz
  const double* h[3];       // widths, length n_a + 1 (last entry 0)
  const double* ih[3];      // 1 / width, last entry 0
  const double* dw[3];      // dual width / mu0 per node, length n_a + 1
};

// Seed-recurrence scalars and per-shift state; lives in device memory and is
// updated only by the single "last" workgroup of a kernel.
struct SolveState {
  double rr;          // (r_k, r_k)
  double rr0;         // (g, g)
  double pAp;         // (p_k, A0 p_k)
  double alpha, beta; // seed alpha_k, beta_k
  double alpha_prev, beta_prev;
  double tol2;        // (rtol * ||g||)^2
  int k;              // seed iteration counter
  int n_active;
  int breakdown;
  int J;
  int B;              // block length
  int pad_;
  double sig_re[kMaxShifts], sig_im[kMaxShifts];    // s_j - s0
  double z_re[kMaxShifts], z_im[kMaxShifts];        // zeta_k
  double zp_re[kMaxShifts], zp_im[kMaxShifts];      // zeta_{k-1}
  int active[kMaxShifts];
  int apply[kMaxShifts];                            // updated at least once in this block
  int iters[kMaxShifts];
  double est[kMaxShifts];                           // |zeta| ||r|| at the stop
  // block coefficients: p_new = a p + sum_l e_l r_l ; y_new = y + c p + sum_l d_l r_l
  double a_re[kMaxShifts], a_im[kMaxShifts];
  double c_re[kMaxShifts], c_im[kMaxShifts];
  double d_re[kMaxShifts][kMaxBlock], d_im[kMaxShifts][kMaxBlock];
  double e_re[kMaxShifts][kMaxBlock], e_im[kMaxShifts][kMaxBlock];
};

struct Reduce {
  double* partials;      // kReduceSlots * kMaxShifts
  unsigned int* counter; // completion counters (zero between kernels)
};

// ---- launchers (tem_kernels.hip) -----------------------------------------
void launch_mass(const GridArgs& g, const double* sigma_cell, double* mass, double* dinv, double* sqrtm,
                 hipStream_t s);
void launch_scale(long long n, const double* a, const double* x, double* y, hipStream_t s);
void launch_to_complex(long long n, const double* x, double2* y, hipStream_t s);
void launch_seed_init(const GridArgs& g, const double* gvec, double* r0, double* pold, double2* Y, double2* P,
                      int J, Reduce red, SolveState* st, hipStream_t s);
void launch_seed_stencil(const GridArgs& g, const double* r, const double* pold, double* pnew, double* q,
                         const double* dinv, double s0, Reduce red, SolveState* st, hipStream_t s);
void launch_seed_update(const GridArgs& g, const double* r, const double* q, double* rnext, Reduce red,
                        SolveState* st, int slot_next, hipStream_t s);
void launch_block_update(const GridArgs& g, const double* R, double2* Y, double2* P, int J, int B,
                         const SolveState* st, hipStream_t s);
void launch_cstencil(const GridArgs& g, const double2* X, long long xstride, const double* dinv,
                     const double* shift_re, const double* shift_im, int nvec, const double2* rhs,
                     double2* out, long long ostride, double* norm_partials, hipStream_t s);
void launch_reduce_rows(const double* partials, int rows, int cols, double* out, hipStream_t s);
void launch_contract(const GridArgs& g, const double2* Y, int J, const double* dinv, const double* C,
                     int T, double* U, hipStream_t s);
void launch_receivers(const GridArgs& g, const double2* Y, int J, const double* dinv, const double* C, int T,
                      const int* rx, int n_rx, int k_s, double* d, hipStream_t s);
void launch_gather_solutions(const GridArgs& g, const double2* Y, int J, const double* dinv, double2* out,
                             hipStream_t s);
void launch_scatter_storage(const GridArgs& g, const double2* xpub, const double* w, double2* xpad, hipStream_t s);
void launch_gather_storage(const GridArgs& g, const double2* xpad, const double* w, double2* xpub, hipStream_t s);
long long storage_edges(const GridArgs& g);
int cstencil_partials(const GridArgs& g);
int reduce_blocks(long long n);

// ---- host RKFIT (tem_rkfit.cpp) --------------------------------------------
struct RkfitResult {
  std::vector<std::complex<double>> xi;      // J poles (pairs with Im > 0, then real)
  std::vector<std::complex<double>> c;       // J * T, factor 2 folded for pairs
  std::vector<double> err;                   // T
};
int rkfit(const std::vector<double>& t, const std::vector<double>& w, int degree, RkfitResult& out,
          std::string& msg);
int table1_degree(double ratio, double tol);

}  // namespace tem
