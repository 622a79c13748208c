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
constexpr int kMaxShifts = 320;  // shifts of one multi-shift solve (the public API takes up to 64 poles)
constexpr int kMaxBlock = 64;       // deferred-update block length (iterations)
constexpr int kReduceSlots = 65536;  // per-kernel partial sums (upper bound on stencil blocks)
// block-coefficient sets: with the block update overlapped with the next
// blocks' seed iterations, block b uses set b mod 3 (and ring third b mod 3)
constexpr int kPhases = 3;

// Node-padded layout: every node (i, j, k), 0 <= i <= nx, ... owns the three
// edges Ex(i,j,k), Ey(i,j,k), Ez(i,j,k) leaving it in +x, +y, +z.  Edges that
// do not exist (Ex at i = nx, ...) and PEC boundary edges are kept as zeros.
// A real field is 3 * nn doubles: component c of node v at c * nn + v, with
// v = (k * py + j) * px + i, px = nx + 1, py = ny + 1.
struct GridArgs {
  int nx, ny, nz;
  int px, py, pz;
  long long nn;             // px * py * pz
  // one allocation of nine arrays of L = max_a n_a + 1 entries: axis a has
  // h[a] = h[0] + 3 a L, ih[a] = h[a] + L, dw[a] = h[a] + 2 L (the seed stencil
  // relies on this layout)
  const double* h[3];       // widths, length n_a + 1 (last entry 0)
  const double* ih[3];      // 1 / width, last entry 0
  const double* dw[3];      // dual width / mu0 per node, length n_a + 1
  int seed_tile = -1;       // seed stencil tile shape (index into the launcher table; host side)
  int step_kz = 2;          // planes per tile of the one-kernel seed step (64 x 8 columns; host side)
};

// Seed-recurrence scalars and per-shift state; lives in device memory.  The
// seed kernels touch only the seed scalars and the per-iteration history;
// the per-shift recurrences are replayed from that history once per block.
struct SolveState {
  // --- read back by the host after every block (keep first) ---
  int k;              // seed iterations done
  int breakdown;
  int J;
  int B;              // block length
  int active[kMaxShifts];
  // --- seed scalars ---
  double rr;          // (r_k, r_k)
  double rr0;         // (g, g)
  double pAp;         // (p_k, A0 p_k)
  double alpha, beta; // alpha_k, beta_k of the last completed steps
  double tol2;        // (rtol ||g||)^2
  double alpha_h[kMaxBlock], beta_h[kMaxBlock], rr_h[kMaxBlock];  // this block's alpha_k, beta_k, (r_{k+1}, r_{k+1})
  double carry_alpha, carry_beta;                                 // alpha, beta of the step before the block
  double rrk[2];                                                  // (r_k, r_k) by parity of k
  // --- per shift ---
  double sig_re[kMaxShifts], sig_im[kMaxShifts];    // s_j - s0
  double z_re[kMaxShifts], z_im[kMaxShifts];        // zeta_k
  double zp_re[kMaxShifts], zp_im[kMaxShifts];      // zeta_{k-1}
  int apply[kPhases][kMaxShifts];                   // updated at least once in this block
  int iters[kMaxShifts];
  double est[kMaxShifts];                           // |zeta| ||r|| at the stop
  // block coefficients: p_new = a p + sum_l e_l r_l ; y_new = y + c p + sum_l d_l r_l,
  // packed per shift for uniform reads: cf[f][j][0] = (a, c), cf[f][j][1 + l] = (e_l, d_l),
  // each complex as (re, im); f is the block's coefficient set
  double cf[kPhases][kMaxShifts][kMaxBlock + 1][4];
};

struct SolveHead {  // the leading part of SolveState
  int k, breakdown, J, B;
  int active[kMaxShifts];
};

// Batched COCG state (adjoint and refinement solves), device memory.
struct CocgState {
  double rho_re[kMaxShifts], rho_im[kMaxShifts];  // r^T r
  double alpha_re[kMaxShifts], alpha_im[kMaxShifts];
  double beta_re[kMaxShifts], beta_im[kMaxShifts];
  double hn2[kMaxShifts];                          // |rhs|^2
  double rn2[kMaxShifts];                          // |r|^2
  double tol2;                                     // rtol^2 (set by the host)
  int cap[kMaxShifts];                             // per-shift iteration cap (set by the host)
  int active[kMaxShifts];
  int iters[kMaxShifts];
  int n_active;
  int breakdown;
  int J;                                           // set by the host
};

// One multi-shift solve in the batched launches of a solve engine: its grid,
// operator and workspace, and where its blocks sit in the batched grids.  The
// seed stencil of every job uses the (64, 8, 1) tile.
struct BatchJob {
  GridArgs g;
  const double* dinv;
  double s0;
  double* R;          // residual ring: B slots of 3 nn
  double* pbuf;       // seed direction, two slots (ping-pong by iteration parity)
  double* q;
  double* part_st;    // stencil partial sums, one per tile
  double* part_up;    // update partial sums
  SolveState* st;
  double2* Y;         // per-shift iterates y_j, J x 3 nn
  double2* P;         // per-shift directions p_j, J x 3 nn
  int J;
  int tile0, ntx, nty, ntiles;  // stencil: first block of this job and its tiles (x, y, total)
  int bu0, nbu;                 // block update: first block and block count
};
constexpr int kMaxBatchJobs = 16;

struct Reduce {
  double* partials;      // kReduceSlots * kMaxShifts
  unsigned int* counter; // completion counters (zero between kernels)
};

// Destination of a solver-block launcher: with graph == nullptr the kernel is
// launched on `stream` at once; otherwise it is appended to `graph` as a
// kernel node depending on node `last` (explicit construction: no stream is
// ever put in capture mode, so device-wide operations issued meanwhile by other
// threads of the process, such as hipFree, cannot invalidate a capture).  The
// first failing node addition is kept in err.
struct Sink {
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphNode_t last = nullptr;
  hipError_t err = hipSuccess;
};

// ---- launchers (tem_kernels.hip) -----------------------------------------
void launch_mass(const GridArgs& g, const double* sigma_cell, double* mass, double* dinv, double* sqrtm,
                 hipStream_t s);
void launch_scale(long long n, const double* a, const double* x, double* y, hipStream_t s);
void launch_to_complex(long long n, const double* x, double2* y, hipStream_t s);
void launch_zero2(long long n, double2* y, hipStream_t s);
void launch_store2(double* p, double a, double b, hipStream_t s);
// r0 = gvec, or r0_scale * gvec (the unscaled seed form's ring)
void launch_seed_init(const GridArgs& g, const double* gvec, double* r0, double* pold, double2* Y, double2* P,
                      int J, Reduce red, SolveState* st, hipStream_t s, const double* r0_scale = nullptr);
void launch_seed_init(const GridArgs& g, const double* gvec, double* r0, double* pold, double2* Y, float2* P,
                      int J, Reduce red, SolveState* st, hipStream_t s, const double* r0_scale = nullptr);
// with t0 != nullptr the dispatch records its own start (t0) and stop (t1) events.
// unscaled (only for the tiles seed_stencil_unscaled_tile accepts): the vectors
// hold M^-1/2 v; the update then gets wd = M^-1/2 to weight (r, r) by M.
bool seed_stencil_unscaled_tile(const GridArgs& g);
void launch_seed_stencil(const GridArgs& g, const double* r, const double* pold, double* pnew, double* q,
                         const double* dinv, double s0, Reduce red, SolveState* st, int local, bool unscaled,
                         Sink& k, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
void launch_seed_update(const GridArgs& g, const double* r, const double* q, double* rnext, Reduce red,
                        SolveState* st, int local, const double* wd, Sink& k, hipEvent_t t0 = nullptr,
                        hipEvent_t t1 = nullptr);
// One-kernel seed step `local` (update of step i fused with the stencil of
// step i + 1): reads r_i, p_i, q_i = A0 p_i, writes r_{i+1} (ring), p_{i+1},
// q_{i+1}; p and q ping-pong by parity (read slot local & 1); partial sums in
// two sets of 4 kReduceSlots entries (red.partials must hold 8 kReduceSlots).
// first != 0: the prologue p_0 = r_0, q_0 = A0 r_0 (pass p = q = r; writes
// slot 0 of p and q).  The vectors (and the ring) hold M^-1/2 v.
void launch_seed_step(const GridArgs& g, const double* r, const double* p, const double* q, double* rn, double* pn,
                      double* qn, const double* dinv, double s0, Reduce red, SolveState* st, int local, int first,
                      Sink& k, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
int seed_step_blocks(const GridArgs& g);
// the shift recurrences after a block of one-kernel seed steps (history complete)
void launch_shift_block_step(const GridArgs& g, int J, Reduce red, SolveState* st, Sink& k, int f = 0);
// R: the block's ring part (slot l holds r_{k0+l}, l = 1 .. B-1), R0: the slot
// holding r_{k0+B}; coefficient set f
// rscale != nullptr: the ring holds M^-1/2 r, scaled back by rscale = M^1/2
void launch_block_update(const GridArgs& g, const double* R, const double* R0, double2* Y, double2* P, int J, int B,
                         const SolveState* st, Sink& k, int f = 0, int max_blocks = 4096,
                         const double* rscale = nullptr);
// precision 1: y_j in FP64, p_j in FP32
void launch_block_update(const GridArgs& g, const double* R, const double* R0, double2* Y, float2* P, int J, int B,
                         const SolveState* st, Sink& k, int f = 0, int max_blocks = 4096,
                         const double* rscale = nullptr);
// J node-padded complex vectors, FP32 storage widened to FP64: sign 0 sets
// Y_j = X_j for all j; sign +1 / -1 adds / subtracts X_j for the j in mask
void launch_accumulate(const GridArgs& g, int J, const float2* X, double2* Y, int sign, unsigned long long mask,
                       hipStream_t s);
void launch_shift_block(const GridArgs& g, int J, Reduce red, SolveState* st, Sink& k, int f = 0);
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
// two-pass form: receiver values and channel contraction straight from the seed residual ring
// (dinv = nullptr: the ring already holds M^-1/2 r)
void launch_ring_receivers(const GridArgs& g, const double* R, int B, const double* dinv, const int* rx, int n_rx,
                           int ks, double* hq, int init, Sink& k);
void launch_ring_contract_init(const GridArgs& g, const double* r0, const double* W, int T, double* U, hipStream_t s);
void launch_ring_contract(const GridArgs& g, const double* R, int B, const double* W, int T, double* U,
                          const SolveState* st, Sink& k);
void launch_ring_fields(const GridArgs& g, const double* U, int T, const double* dinv, double* fields,
                        const int* rx, int n_rx, int ks, double* d, hipStream_t s);
long long storage_edges(const GridArgs& g);
int cstencil_partials(const GridArgs& g);
int seed_stencil_blocks(const GridArgs& g);
// seed stencil tile shape for a grid on a device with n_cu compute units
int choose_seed_tile(const GridArgs& g, int n_cu);
// batched launches of a solve engine: every job's blocks in one grid per kernel
int batch_tiles(const GridArgs& g, int* ntx, int* nty);  // (64, 8, 1) tiles of a grid
int block_update_blocks(const GridArgs& g);
void launch_seed_stencil_batch(const BatchJob* jobs, int njobs, int total_tiles, int B, int local, Sink& k);
void launch_seed_update_batch(const BatchJob* jobs, int njobs, int B, int local, Sink& k);
void launch_shift_block_batch(const BatchJob* jobs, int njobs, int max_J, Sink& k);
void launch_block_update_batch(const BatchJob* jobs, int njobs, int total_blocks, int B, Sink& k);
void launch_gather_heads(const BatchJob* jobs, int njobs, SolveHead* out, Sink& k);
// adjoint: batched COCG (state is an opaque device struct of cocg_state_bytes())
size_t cocg_state_bytes();
int cocg_partials(const GridArgs& g, int J);
void launch_adj_rhs(const GridArgs& g, int J, int n_rx, const int* rx, int ks, const double* gamma, const double* dinv,
                    double2* H, hipStream_t s);
void launch_cocg_init(const GridArgs& g, int J, const double2* H, double2* Mu, double2* Rr, double2* Pold,
                      double* partials, unsigned int* counter, void* st, hipStream_t s);
void launch_cocg_stencil(const GridArgs& g, int J, const double2* Rr, const double2* Pold, double2* Pnew, double2* Q,
                         const double* dinv, const double* sre, const double* sim, double* partials,
                         unsigned int* counter, void* st, hipStream_t s);
void launch_cocg_update(const GridArgs& g, int J, double2* Mu, double2* Rr, const double2* Pn, const double2* Q,
                        double* partials, unsigned int* counter, void* st, hipStream_t s);
// the same batched COCG with complex FP32 vector storage (FP64 scalars and dot products)
void launch_cocg_init(const GridArgs& g, int J, const double2* H, float2* Mu, float2* Rr, float2* Pold,
                      double* partials, unsigned int* counter, void* st, hipStream_t s);
void launch_cocg_stencil(const GridArgs& g, int J, const float2* Rr, const float2* Pold, float2* Pnew, float2* Q,
                         const double* dinv, const double* sre, const double* sim, double* partials,
                         unsigned int* counter, void* st, hipStream_t s);
void launch_cocg_update(const GridArgs& g, int J, float2* Mu, float2* Rr, const float2* Pn, const float2* Q,
                        double* partials, unsigned int* counter, void* st, hipStream_t s);
void launch_grad_edges(const GridArgs& g, int J, const double2* Mu, const double2* Y, const double* dinv,
                       const double* sre, const double* sim, double* z, hipStream_t s);
void launch_grad_cells(const GridArgs& g, const double* sigma, const double* z, double* grad, hipStream_t s);
// Jacobian action: h_j = -s_j (dM/M) y_j with dM the edge mass of dm_c sigma_c (per cell)
void launch_jvp_rhs(const GridArgs& g, int J, const double* sigma, const double* dm, const double* mass,
                    const double* sre, const double* sim, const double2* Y, double2* H, hipStream_t s);
void launch_caxpy_shifts(const GridArgs& g, int J, const double* gamma, const double2* Yr, double2* Mu,
                         hipStream_t s);
// per shift (w_j, rho_j) (Hermitian, re and im) and (w_j, w_j): partial sums at
// partials[(3 j + m) * dot_shifts_blocks(g) + block], m = 0, 1, 2
int dot_shifts_blocks(const GridArgs& g);
void launch_dot_shifts(const GridArgs& g, int J, const double2* W, const double2* Rh, double* partials, hipStream_t s);

// ---- host RKFIT (tem_rkfit.cpp) --------------------------------------------
struct RkfitResult {
  std::vector<std::complex<double>> xi;      // J poles (pairs with Im > 0, then real)
  std::vector<std::complex<double>> c;       // J * T, factor 2 folded for pairs
  std::vector<double> err;                   // T
};
int rkfit(const std::vector<double>& t, const std::vector<double>& w, int degree, RkfitResult& out,
          std::string& msg);
int table1_degree(double ratio, double tol);
// single-time best approximation of exp(-x) of type [m/m] (Sec. 3.1)
struct SingleResult {
  std::vector<std::complex<double>> xi;  // ceil(m/2) poles (pairs with Im > 0, then real)
  std::vector<std::complex<double>> a;   // residues, factor 2 folded for pairs
  double a0 = 0.0;                       // constant term
  double err = 0.0;                      // uniform error on [0, inf)
};
int best_rational(int m, SingleResult& out, std::string& msg);

}  // namespace tem
