// Host RKFIT for the shared-pole family of Sec. 3.2, eq. (ratfam):
//   r^[k](x) = sum_i alpha_i^[k] / (x - xi_i)  ~  exp(-t_k x),  x >= 0,
// type [(m-1)/m], poles shared by every channel.  RKFIT minimizes eq.
// (rkfit), sum_k w_k || r^[k](S) v - exp(-t_k S) v ||^2, for a diagonal
// surrogate S with dense eigenvalues on [0, inf) and v = ones, by implicit
// pole relocation (Berljafa & Guettel, cited in Sec. 3.2):
//   1. orthonormal rational Krylov basis V of Q_{m+1}(S, v, q_m) with the
//      current poles (rational Arnoldi), with its pencil S V K = V H;
//   2. the unit c minimizing sum_k w_k ||(I - V V^*) F_k V c||^2 (smallest
//      right singular vector of the stacked matrix, F_k = exp(-t_k S));
//   3. the new poles: eigenvalues of the trailing m x m part of the pencil
//      (Q^* H, Q^* K), Q unitary with first column c.
// Residues: real least squares over {1/(x - xi_i)} per channel.
//
// Choices the paper leaves open (they match the oracle's reading of the
// same passage, implemented independently): surrogate = 0 and 2000
// log-spaced points on [1e-3, 1e4/tau_min] in tau = t/t_max; start poles
// -r e^{+-i pi/3}, r log-spaced on [1, 1/tau_min]; 20 sweeps keeping the
// sweep with the smallest (weighted, eq. (uniform_error)) uniform error on a coarse check set; relocated
// poles symmetrized into conjugate pairs, a real pole on x >= 0 reflected.
//
// Dense kernels (all hand-written; no LAPACK is linked): Householder QR,
// one-sided Jacobi SVD, LU with partial pivoting, Hessenberg reduction and
// the shifted complex QR algorithm for eigenvalues.
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tem.h"
#include "tem_internal.h"

namespace tem {
namespace {

using cd = std::complex<double>;

// Column-major dense complex matrix.
struct Mat {
  int m = 0, n = 0;
  std::vector<cd> a;
  Mat() = default;
  Mat(int m_, int n_) : m(m_), n(n_), a((size_t)m_ * n_, cd(0.0, 0.0)) {}
  cd& operator()(int i, int j) { return a[(size_t)j * m + i]; }
  const cd& operator()(int i, int j) const { return a[(size_t)j * m + i]; }
  cd* col(int j) { return &a[(size_t)j * m]; }
  const cd* col(int j) const { return &a[(size_t)j * m]; }
};

double nrm2(const cd* x, int n) {
  double s = 0.0, scale = 0.0;
  for (int i = 0; i < n; ++i) scale = std::max(scale, std::abs(x[i]));
  if (scale == 0.0) return 0.0;
  for (int i = 0; i < n; ++i) s += std::norm(x[i] / scale);
  return scale * std::sqrt(s);
}

// In-place Householder QR of A (m >= n); returns the n x n R.
Mat householder_r(Mat A) {
  const int m = A.m, n = A.n;
  std::vector<cd> v(m);
  for (int c = 0; c < n && c < m; ++c) {
    cd* x = A.col(c) + c;
    const int len = m - c;
    const double xn = nrm2(x, len);
    if (xn == 0.0) continue;
    const cd ph = std::abs(x[0]) > 0.0 ? x[0] / std::abs(x[0]) : cd(1.0, 0.0);
    const cd alpha = -ph * xn;
    for (int i = 0; i < len; ++i) v[i] = x[i];
    v[0] -= alpha;
    const double vn = nrm2(v.data(), len);
    if (vn == 0.0) continue;
    for (int i = 0; i < len; ++i) v[i] /= vn;
    for (int j = c; j < n; ++j) {
      cd* y = A.col(j) + c;
      cd d(0.0, 0.0);
      for (int i = 0; i < len; ++i) d += std::conj(v[i]) * y[i];
      d *= 2.0;
      for (int i = 0; i < len; ++i) y[i] -= d * v[i];
    }
  }
  Mat R(n, n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j && i < m; ++i) R(i, j) = A(i, j);
  return R;
}

// Right singular vector of the smallest singular value (one-sided Jacobi).
std::vector<cd> smallest_right_singular(const Mat& R0) {
  Mat W = R0;
  const int n = W.n;
  Mat V(n, n);
  for (int i = 0; i < n; ++i) V(i, i) = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double a = 0.0, b = 0.0;
        cd g(0.0, 0.0);
        const cd* wp = W.col(p);
        const cd* wq = W.col(q);
        for (int i = 0; i < W.m; ++i) {
          a += std::norm(wp[i]);
          b += std::norm(wq[i]);
          g += std::conj(wp[i]) * wq[i];
        }
        const double ag = std::abs(g);
        if (ag == 0.0 || ag <= 1e-15 * std::sqrt(a * b)) continue;
        off = std::max(off, ag / std::sqrt(a * b));
        const cd ph = std::conj(g) / ag;  // q' = q * conj(g)/|g| makes p^H q' = |g|
        const double zeta = (b - a) / (2.0 * ag);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::abs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (Mat* M : {&W, &V}) {
          cd* mp = M->col(p);
          cd* mq = M->col(q);
          for (int i = 0; i < M->m; ++i) {
            const cd x = mp[i], y = mq[i] * ph;
            mp[i] = cs * x - sn * y;
            mq[i] = sn * x + cs * y;
          }
        }
      }
    }
    if (off < 1e-15) break;
  }
  int best = 0;
  double bn = 1e300;
  for (int j = 0; j < n; ++j) {
    const double s = nrm2(W.col(j), W.m);
    if (s < bn) {
      bn = s;
      best = j;
    }
  }
  return std::vector<cd>(V.col(best), V.col(best) + n);
}

// Solve A X = B in place (A n x n, LU with partial pivoting); false if singular.
bool lu_solve(Mat A, Mat& B) {
  const int n = A.n;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A(i, k)) > std::abs(A(piv, k))) piv = i;
    if (std::abs(A(piv, k)) == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A(k, j), A(piv, j));
      for (int j = 0; j < B.n; ++j) std::swap(B(k, j), B(piv, j));
    }
    for (int i = k + 1; i < n; ++i) {
      const cd f = A(i, k) / A(k, k);
      if (f == cd(0.0, 0.0)) continue;
      for (int j = k; j < n; ++j) A(i, j) -= f * A(k, j);
      for (int j = 0; j < B.n; ++j) B(i, j) -= f * B(k, j);
    }
  }
  for (int j = 0; j < B.n; ++j)
    for (int i = n - 1; i >= 0; --i) {
      cd s = B(i, j);
      for (int l = i + 1; l < n; ++l) s -= A(i, l) * B(l, j);
      B(i, j) = s / A(i, i);
    }
  return true;
}

// Eigenvalues of a general complex matrix: Householder reduction to upper
// Hessenberg form, then the explicitly shifted QR algorithm with Givens
// rotations, Wilkinson shifts and deflation on negligible subdiagonals.
bool eigenvalues(Mat H, std::vector<cd>& ev) {
  const int n = H.n;
  std::vector<cd> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    cd* x = &H(k + 1, k);
    std::vector<cd> xs(len);
    for (int i = 0; i < len; ++i) xs[i] = H(k + 1 + i, k);
    const double xn = nrm2(xs.data(), len);
    if (xn == 0.0) continue;
    (void)x;
    const cd ph = std::abs(xs[0]) > 0 ? xs[0] / std::abs(xs[0]) : cd(1.0, 0.0);
    for (int i = 0; i < len; ++i) v[i] = xs[i];
    v[0] += ph * xn;
    const double vn = nrm2(v.data(), len);
    for (int i = 0; i < len; ++i) v[i] /= vn;
    for (int j = 0; j < n; ++j) {  // H <- (I - 2vv^*) H
      cd d(0.0, 0.0);
      for (int i = 0; i < len; ++i) d += std::conj(v[i]) * H(k + 1 + i, j);
      d *= 2.0;
      for (int i = 0; i < len; ++i) H(k + 1 + i, j) -= d * v[i];
    }
    for (int i = 0; i < n; ++i) {  // H <- H (I - 2vv^*)
      cd d(0.0, 0.0);
      for (int l = 0; l < len; ++l) d += H(i, k + 1 + l) * v[l];
      d *= 2.0;
      for (int l = 0; l < len; ++l) H(i, k + 1 + l) -= d * std::conj(v[l]);
    }
    for (int i = k + 2; i < n; ++i) H(i, k) = 0.0;
  }
  ev.assign(n, cd(0.0, 0.0));
  int hi = n - 1;
  int iter = 0, total = 0;
  const double eps = 2.2e-16;
  std::vector<double> cs(n);
  std::vector<cd> sn(n);
  while (hi >= 0) {
    if (hi == 0) {
      ev[0] = H(0, 0);
      break;
    }
    int lo = hi;
    while (lo > 0) {
      const double t = std::abs(H(lo, lo)) + std::abs(H(lo - 1, lo - 1));
      if (std::abs(H(lo, lo - 1)) <= eps * (t > 0 ? t : 1.0)) break;
      --lo;
    }
    if (lo == hi) {
      ev[hi] = H(hi, hi);
      --hi;
      iter = 0;
      continue;
    }
    if (++total > 100 * n) return false;
    ++iter;
    // Wilkinson shift from the trailing 2x2 block
    const cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
    const cd tr = a + d, det = a * d - b * c;
    const cd disc = std::sqrt(tr * tr - 4.0 * det);
    const cd l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
    cd mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
    if (iter % 11 == 10) mu = d + std::abs(H(hi, hi - 1)) * cd(0.75, 0.5);  // exceptional shift
    for (int i = lo; i <= hi; ++i) H(i, i) -= mu;
    for (int k = lo; k < hi; ++k) {
      const cd x = H(k, k), y = H(k + 1, k);
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      double cc;
      cd ss;
      if (r == 0.0) {
        cc = 1.0;
        ss = 0.0;
      } else if (std::abs(x) == 0.0) {
        cc = 0.0;
        ss = 1.0;
      } else {
        cc = std::abs(x) / r;
        ss = x * std::conj(y) / (std::abs(x) * r);
      }
      cs[k] = cc;
      sn[k] = ss;
      for (int j = k; j <= hi; ++j) {  // rows k, k+1 <- G rows
        const cd p = H(k, j), q = H(k + 1, j);
        H(k, j) = cc * p + ss * q;
        H(k + 1, j) = -std::conj(ss) * p + cc * q;
      }
    }
    for (int k = lo; k < hi; ++k) {  // columns k, k+1 <- cols G^H
      const double cc = cs[k];
      const cd ss = sn[k];
      for (int i = lo; i <= std::min(k + 2, hi); ++i) {
        const cd p = H(i, k), q = H(i, k + 1);
        H(i, k) = cc * p + std::conj(ss) * q;
        H(i, k + 1) = -ss * p + cc * q;
      }
    }
    for (int i = lo; i <= hi; ++i) H(i, i) += mu;
  }
  return true;
}

// Rational Arnoldi on the diagonal surrogate x with the unit starting vector
// v0 and the poles: orthonormal V (N x m+1) and the (m+1) x m pencil with
// S V Kp = V Hp.  Step j solves (S - xi_j) w = v_j, orthogonalizes twice
// (classical Gram-Schmidt) and normalizes; false on breakdown.
bool rational_arnoldi(const std::vector<double>& x, const std::vector<double>& v0, const std::vector<cd>& poles,
                      Mat& V, Mat& Kp, Mat& Hp) {
  const int N = (int)x.size(), m = (int)poles.size();
  V = Mat(N, m + 1);
  Kp = Mat(m + 1, m);
  Hp = Mat(m + 1, m);
  for (int i = 0; i < N; ++i) V(i, 0) = v0[i];
  std::vector<cd> wv(N), h(m + 1);
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < N; ++i) wv[i] = V(i, j) / (x[i] - poles[j]);
    std::vector<cd> kc(j + 2, cd(0.0, 0.0));
    for (int pass = 0; pass < 2; ++pass) {
      for (int l = 0; l <= j; ++l) {
        cd d(0.0, 0.0);
        const cd* vl = V.col(l);
        for (int i = 0; i < N; ++i) d += std::conj(vl[i]) * wv[i];
        h[l] = d;
      }
      for (int l = 0; l <= j; ++l) {
        const cd* vl = V.col(l);
        for (int i = 0; i < N; ++i) wv[i] -= h[l] * vl[i];
        kc[l] += h[l];
      }
    }
    kc[j + 1] = nrm2(wv.data(), N);
    if (kc[j + 1] == cd(0.0, 0.0)) return false;
    for (int i = 0; i < N; ++i) V(i, j + 1) = wv[i] / kc[j + 1];
    for (int l = 0; l <= j + 1; ++l) {
      Kp(l, j) = kc[l];
      Hp(l, j) = poles[j] * kc[l];
    }
    Hp(j, j) += 1.0;
  }
  return true;
}

// RKFIT's new poles for the unit coefficient vector c: with the Householder
// Q whose first column is c (up to a phase), the eigenvalues of the trailing
// m x m part of the pencil (Q^* Hp, Q^* Kp).  False if the pencil is singular
// or the QR iteration does not converge.
bool relocated_poles(const Mat& Hp, const Mat& Kp, const std::vector<cd>& c, std::vector<cd>& z) {
  const int m1 = (int)c.size(), m = m1 - 1;
  std::vector<cd> u(c);
  const cd ph = std::abs(c[0]) > 0 ? c[0] / std::abs(c[0]) : cd(1.0, 0.0);
  u[0] += ph;  // u = c - alpha e1 with alpha = -ph (|c| = 1)
  const double un = nrm2(u.data(), m1);
  for (auto& e : u) e /= un;
  auto reflect = [&](const Mat& P) {  // (I - 2 u u^*) P
    Mat Q = P;
    for (int j = 0; j < P.n; ++j) {
      cd d(0.0, 0.0);
      for (int i = 0; i < m1; ++i) d += std::conj(u[i]) * P(i, j);
      d *= 2.0;
      for (int i = 0; i < m1; ++i) Q(i, j) -= d * u[i];
    }
    return Q;
  };
  const Mat Ht = reflect(Hp), Kt = reflect(Kp);
  Mat A(m, m), Bm(m, m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      A(i, j) = Ht(i + 1, j);
      Bm(i, j) = Kt(i + 1, j);
    }
  return lu_solve(Bm, A) && eigenvalues(A, z);
}

struct Fit {
  std::vector<cd> reps;  // pairs (Im > 0) then real
  std::vector<cd> A;     // J x K residues (row j: A[j*K + k])
};

std::vector<cd> symmetrize(std::vector<cd> z, const std::vector<cd>& prev) {
  const double rel = 1e-10;
  for (size_t i = 0; i < z.size(); ++i)
    if (!std::isfinite(z[i].real()) || !std::isfinite(z[i].imag())) z[i] = prev[i % prev.size()];
  std::vector<cd> up, lo;
  std::vector<double> reals;
  for (const cd& p : z) {
    if (std::abs(p.imag()) <= rel * std::abs(p)) reals.push_back(p.real());
    else if (p.imag() > 0) up.push_back(p);
    else lo.push_back(std::conj(p));
  }
  std::vector<cd> out;
  while (!up.empty() && !lo.empty()) {
    size_t bi = 0, bj = 0;
    double bd = 1e300;
    for (size_t i = 0; i < up.size(); ++i)
      for (size_t j = 0; j < lo.size(); ++j) {
        const double d = std::abs(up[i] - lo[j]);
        if (d < bd) {
          bd = d;
          bi = i;
          bj = j;
        }
      }
    const cd p = 0.5 * (up[bi] + lo[bj]);
    out.push_back(p);
    out.push_back(std::conj(p));
    up.erase(up.begin() + bi);
    lo.erase(lo.begin() + bj);
  }
  for (const cd& p : up) reals.push_back(p.real());
  for (const cd& p : lo) reals.push_back(p.real());
  for (double r : reals) out.push_back(cd(r >= 0 ? -std::abs(r) - 0.0 : r, 0.0));
  for (cd& p : out)
    if (p.imag() == 0.0 && p.real() == 0.0) p = cd(-1e-6, 0.0);
  return out;
}

std::vector<cd> representatives(const std::vector<cd>& poles) {
  std::vector<cd> up, re;
  for (const cd& p : poles) {
    if (p.imag() > 0) up.push_back(p);
    else if (p.imag() == 0) re.push_back(p);
  }
  auto by_abs = [](const cd& a, const cd& b) { return std::abs(a) < std::abs(b); };
  std::sort(up.begin(), up.end(), by_abs);
  std::sort(re.begin(), re.end(), by_abs);
  up.insert(up.end(), re.begin(), re.end());
  return up;
}

// Real least-squares residues for every channel over the subdiagonal basis.
std::vector<cd> fit_residues(const std::vector<cd>& reps, const std::vector<double>& tau,
                             const std::vector<double>& x) {
  const int N = (int)x.size(), K = (int)tau.size();
  int ncol = 0;
  for (const cd& p : reps) ncol += p.imag() > 0 ? 2 : 1;
  // real matrix stored as complex with zero imaginary parts (reuse the QR)
  Mat B(N, ncol + K);
  std::vector<double> scale(ncol);
  int col = 0;
  for (const cd& p : reps) {
    if (p.imag() > 0) {
      for (int i = 0; i < N; ++i) {
        const cd g = 1.0 / (x[i] - p);
        B(i, col) = 2.0 * g.real();
        B(i, col + 1) = -2.0 * g.imag();
      }
      col += 2;
    } else {
      for (int i = 0; i < N; ++i) B(i, col) = (1.0 / (x[i] - p)).real();
      col += 1;
    }
  }
  for (int j = 0; j < ncol; ++j) {
    scale[j] = nrm2(B.col(j), N);
    if (scale[j] == 0.0) scale[j] = 1.0;
    for (int i = 0; i < N; ++i) B(i, j) /= scale[j];
  }
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < N; ++i) B(i, ncol + k) = std::exp(-tau[k] * x[i]);
  // QR of [B | Y]: the leading ncol x ncol block is R, the next columns Q^T Y
  Mat R = householder_r(B);
  std::vector<cd> Aout(reps.size() * (size_t)K);
  std::vector<double> coef(ncol);
  for (int k = 0; k < K; ++k) {
    for (int i = ncol - 1; i >= 0; --i) {
      double s = R(i, ncol + k).real();
      for (int l = i + 1; l < ncol; ++l) s -= R(i, l).real() * coef[l];
      const double d = R(i, i).real();
      coef[i] = d != 0.0 ? s / d : 0.0;
    }
    int r = 0;
    for (size_t j = 0; j < reps.size(); ++j) {
      if (reps[j].imag() > 0) {
        Aout[j * K + k] = cd(coef[r] / scale[r], coef[r + 1] / scale[r + 1]);
        r += 2;
      } else {
        Aout[j * K + k] = cd(coef[r] / scale[r], 0.0);
        r += 1;
      }
    }
  }
  return Aout;
}

// eq. (error) on a log-spaced check set plus the |sum of residues|/x tail.
std::vector<double> channel_errors(const std::vector<cd>& reps, const std::vector<cd>& A,
                                   const std::vector<double>& tau, int npts) {
  const int K = (int)tau.size();
  const double tmin = *std::min_element(tau.begin(), tau.end());
  const double lo = -6.0, hi = std::log10(1e8 / tmin);
  const int nth = std::max(1, std::min(8, (int)std::thread::hardware_concurrency()));
  std::vector<std::vector<double>> part(nth, std::vector<double>(K, 0.0));
  auto work = [&](int t) {
    std::vector<double> r(K);
    for (int i = t; i <= npts; i += nth) {
      const double x = i == 0 ? 0.0 : std::pow(10.0, lo + (hi - lo) * (i - 1) / (npts - 1));
      std::fill(r.begin(), r.end(), 0.0);
      for (size_t j = 0; j < reps.size(); ++j) {
        const cd g = 1.0 / (x - reps[j]);
        const bool pr = reps[j].imag() > 0;
        for (int k = 0; k < K; ++k) {
          const double v = (A[j * K + k] * g).real();
          r[k] += pr ? 2.0 * v : v;
        }
      }
      for (int k = 0; k < K; ++k) part[t][k] = std::max(part[t][k], std::abs(std::exp(-tau[k] * x) - r[k]));
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nth; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& x : th) x.join();
  std::vector<double> err(K, 0.0);
  const double xmax = std::pow(10.0, hi);
  for (int k = 0; k < K; ++k) {
    double lead = 0.0;
    for (size_t j = 0; j < reps.size(); ++j) lead += (reps[j].imag() > 0 ? 2.0 : 1.0) * A[j * K + k].real();
    err[k] = std::abs(lead) / xmax;
    for (int t = 0; t < nth; ++t) err[k] = std::max(err[k], part[t][k]);
  }
  return err;
}

}  // namespace

int table1_degree(double ratio, double tol) {
  // Table 1: degree for accuracy tol over [t_min, t_max] (columns: ratio)
  static const double ratios[6] = {1.0, 1e1, 1e2, 1e3, 1e4, 1e5};
  static const double tols[5] = {1e-2, 1e-4, 1e-6, 1e-8, 1e-10};
  static const int deg[5][6] = {{2, 5, 7, 10, 12, 14},
                                {4, 9, 14, 18, 22, 26},
                                {7, 14, 20, 27, 33, 38},
                                {9, 18, 27, 35, 44, 52},
                                {11, 23, 33, 44, 54, 63}};
  int c = -1, r = -1;
  for (int i = 0; i < 6; ++i)
    if (ratios[i] >= ratio * (1 - 1e-12)) {
      c = i;
      break;
    }
  for (int i = 0; i < 5; ++i)
    if (tols[i] <= tol * (1 + 1e-12)) {
      r = i;
      break;
    }
  if (c < 0 || r < 0) return -1;
  int d = deg[r][c];
  return d + (d & 1);  // even, so that the poles pair up
}

int rkfit(const std::vector<double>& t, const std::vector<double>& w, int m, RkfitResult& out, std::string& msg) {
  const int K = (int)t.size();
  const double tmax = *std::max_element(t.begin(), t.end());
  std::vector<double> tau(K);
  for (int k = 0; k < K; ++k) tau[k] = t[k] / tmax;
  const double tmin = *std::min_element(tau.begin(), tau.end());
  // surrogate eigenvalues
  const int ns = 2000;
  std::vector<double> x(ns + 1);
  x[0] = 0.0;
  const double l0 = -3.0, l1 = std::log10(1e4 / tmin);
  for (int i = 0; i < ns; ++i) x[i + 1] = std::pow(10.0, l0 + (l1 - l0) * i / (ns - 1));
  const int N = ns + 1;
  // start poles
  std::vector<cd> poles;
  const int np = m / 2;
  for (int i = 0; i < np; ++i) {
    const double r = np > 1 ? std::pow(10.0, std::log10(1.0 / tmin) * i / (np - 1)) : 1.0;
    poles.push_back(-r * std::exp(cd(0.0, M_PI / 3)));
  }
  for (int i = 0; i < np; ++i) poles.push_back(std::conj(poles[i]));
  if (m % 2) poles.push_back(cd(-1.0 / std::sqrt(tmin), 0.0));

  const std::vector<double> v0(N, 1.0 / std::sqrt((double)N));  // v = ones, normalized

  double best_err = 1e300;
  Fit best;
  const int nth = std::max(1, std::min(8, (int)std::thread::hardware_concurrency()));
  for (int sweep = 0; sweep < 20; ++sweep) {
    // 1. rational Arnoldi
    Mat V, Kp, Hp;
    if (!rational_arnoldi(x, v0, poles, V, Kp, Hp)) {
      msg = "rational Arnoldi breakdown";
      return TEM_EBREAKDOWN;
    }
    // 2. stacked (I - V V^*) F_k V, reduced to R per thread (TSQR), then combined
    const int m1 = m + 1;
    std::vector<Mat> Rs(nth);
    auto work = [&](int tid) {
      Mat acc;
      bool have = false;
      for (int k = tid; k < K; k += nth) {
        Mat L(N + (have ? m1 : 0), m1);
        Mat FV(N, m1);
        for (int j = 0; j < m1; ++j)
          for (int i = 0; i < N; ++i) FV(i, j) = std::exp(-tau[k] * x[i]) * V(i, j);
        Mat G(m1, m1);
        for (int j = 0; j < m1; ++j)
          for (int l = 0; l < m1; ++l) {
            cd d(0.0, 0.0);
            const cd* vl = V.col(l);
            const cd* fj = FV.col(j);
            for (int i = 0; i < N; ++i) d += std::conj(vl[i]) * fj[i];
            G(l, j) = d;
          }
        const double sw = std::sqrt(w[k]);
        for (int j = 0; j < m1; ++j) {
          for (int i = 0; i < N; ++i) {
            cd s = FV(i, j);
            for (int l = 0; l < m1; ++l) s -= V(i, l) * G(l, j);
            L(i, j) = sw * s;
          }
          if (have)
            for (int i = 0; i < m1; ++i) L(N + i, j) = acc(i, j);
        }
        acc = householder_r(L);
        have = true;
      }
      if (!have) acc = Mat(m1, m1);
      Rs[tid] = acc;
    };
    std::vector<std::thread> th;
    for (int tid = 1; tid < nth; ++tid) th.emplace_back(work, tid);
    work(0);
    for (auto& tt : th) tt.join();
    Mat Stack(nth * m1, m1);
    for (int tid = 0; tid < nth; ++tid)
      for (int j = 0; j < m1; ++j)
        for (int i = 0; i < m1; ++i) Stack(tid * m1 + i, j) = Rs[tid](i, j);
    const Mat R = householder_r(Stack);
    std::vector<cd> c = smallest_right_singular(R);
    // 3. new poles from the trailing pencil
    std::vector<cd> z;
    if (!relocated_poles(Hp, Kp, c, z)) {
      msg = "pole relocation failed (singular pencil or no QR convergence)";
      if (best.reps.empty()) return TEM_EBREAKDOWN;
      break;
    }
    poles = symmetrize(z, poles);
    const std::vector<cd> reps = representatives(poles);
    const std::vector<cd> Ares = fit_residues(reps, tau, x);
    // eq. (uniform_error): the weighted maximum over the channels (all weights 1
    // gives the plain uniform error)
    const std::vector<double> e = channel_errors(reps, Ares, tau, 4000);
    double emax = 0.0;
    for (size_t k = 0; k < e.size(); ++k) emax = std::max(emax, w[k] * e[k]);
    if (std::isfinite(emax) && emax < best_err) {
      best_err = emax;
      best.reps = reps;
      best.A = Ares;
    }
  }
  if (best.reps.empty()) {
    msg = "RKFIT produced no finite fit";
    return TEM_EBREAKDOWN;
  }
  const std::vector<double> err = channel_errors(best.reps, best.A, tau, 200000);
  const int J = (int)best.reps.size();
  out.xi.resize(J);
  out.c.resize((size_t)J * K);
  out.err = err;
  for (int j = 0; j < J; ++j) {
    out.xi[j] = best.reps[j] / tmax;
    const double f = best.reps[j].imag() > 0 ? 2.0 : 1.0;
    for (int k = 0; k < K; ++k) out.c[(size_t)j * K + k] = f * best.A[(size_t)j * K + k] / tmax;
  }
  return TEM_OK;
}

// Single-time best approximation (Sec. 3.1): the type-[m/m] function
//   r(x) = a0 + sum_i alpha_i / (x - xi_i)  ~  exp(-x)  on [0, inf)
// with the smallest uniform error.  The paper takes it from the literature
// without a method; here RKFIT relocates the poles on the one channel t = 1
// with a constant term in the residue fit, and Lawson's iteratively
// reweighted least squares turns the least-squares fit into the minimax one:
// after 5 unweighted sweeps, every sweep multiplies the sample weights by
// |error|^(1/2) (normalized to max 1) and relocates in the weighted inner
// product (starting vector sqrt(w)).  80 sweeps; the one with the smallest
// uniform error is kept.  Samples: 0 and 9 (1 + s)/(1 - s) at Chebyshev
// points s = -cos(pi l / 1999) < 1.
namespace {

// weighted least-squares a0 and residues (pairs: one complex residue, real
// poles: a real one) over the constant and {1/(x - p)}
void fit_with_constant(const std::vector<cd>& reps, const std::vector<double>& x, const std::vector<double>& y,
                       const std::vector<double>& w, double& a0, std::vector<cd>& alpha) {
  const int N = (int)x.size();
  int ncol = 1;
  for (const cd& p : reps) ncol += p.imag() > 0 ? 2 : 1;
  Mat B(N, ncol + 1);
  std::vector<double> sw(N);
  for (int i = 0; i < N; ++i) sw[i] = std::sqrt(w[i]);
  for (int i = 0; i < N; ++i) B(i, 0) = sw[i];
  int col = 1;
  for (const cd& p : reps) {
    for (int i = 0; i < N; ++i) {
      const cd g = 1.0 / (x[i] - p);
      if (p.imag() > 0) {
        B(i, col) = sw[i] * 2.0 * g.real();
        B(i, col + 1) = -sw[i] * 2.0 * g.imag();
      } else {
        B(i, col) = sw[i] * g.real();
      }
    }
    col += p.imag() > 0 ? 2 : 1;
  }
  std::vector<double> scale(ncol);
  for (int j = 0; j < ncol; ++j) {
    scale[j] = nrm2(B.col(j), N);
    if (scale[j] == 0.0) scale[j] = 1.0;
    for (int i = 0; i < N; ++i) B(i, j) /= scale[j];
  }
  for (int i = 0; i < N; ++i) B(i, ncol) = sw[i] * y[i];
  const Mat R = householder_r(B);
  std::vector<double> coef(ncol);
  for (int i = ncol - 1; i >= 0; --i) {
    double s = R(i, ncol).real();
    for (int l = i + 1; l < ncol; ++l) s -= R(i, l).real() * coef[l];
    const double d = R(i, i).real();
    coef[i] = d != 0.0 ? s / d : 0.0;
  }
  for (int j = 0; j < ncol; ++j) coef[j] /= scale[j];
  a0 = coef[0];
  alpha.assign(reps.size(), cd(0.0, 0.0));
  int r = 1;
  for (size_t j = 0; j < reps.size(); ++j) {
    if (reps[j].imag() > 0) {
      alpha[j] = cd(coef[r], coef[r + 1]);
      r += 2;
    } else {
      alpha[j] = cd(coef[r], 0.0);
      r += 1;
    }
  }
}

double eval_single(const std::vector<cd>& reps, const std::vector<cd>& alpha, double a0, double x) {
  double r = a0;
  for (size_t j = 0; j < reps.size(); ++j) {
    const double v = (alpha[j] / (x - reps[j])).real();
    r += reps[j].imag() > 0 ? 2.0 * v : v;
  }
  return r;
}

// max |exp(-x) - r(x)| over 0, npts log-spaced points on [1e-6, 1e8] and
// x = infinity (where r = a0)
double single_error(const std::vector<cd>& reps, const std::vector<cd>& alpha, double a0, int npts) {
  const int nth = std::max(1, std::min(8, (int)std::thread::hardware_concurrency()));
  std::vector<double> part(nth, 0.0);
  auto work = [&](int t) {
    for (int i = t; i <= npts; i += nth) {
      const double x = i == 0 ? 0.0 : std::pow(10.0, -6.0 + 14.0 * (i - 1) / (npts - 1));
      part[t] = std::max(part[t], std::abs(std::exp(-x) - eval_single(reps, alpha, a0, x)));
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nth; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& t : th) t.join();
  double e = std::abs(a0);
  for (double p : part) e = std::max(e, p);
  return e;
}

}  // namespace

int best_rational(int m, SingleResult& out, std::string& msg) {
  std::vector<double> x{0.0};
  const int ns = 2000;
  for (int l = 1; l < ns; ++l) {
    const double s = -std::cos(M_PI * l / (ns - 1));
    if (s < 1.0) x.push_back(9.0 * (1.0 + s) / (1.0 - s));
  }
  const int N = (int)x.size();
  std::vector<double> y(N), w(N, 1.0), v0(N);
  for (int i = 0; i < N; ++i) y[i] = std::exp(-x[i]);
  std::vector<cd> poles;
  for (int i = 0; i < m / 2; ++i) poles.push_back(-std::exp(cd(0.0, M_PI / 3)));
  for (int i = 0; i < m / 2; ++i) poles.push_back(-std::exp(cd(0.0, -M_PI / 3)));
  if (m % 2) poles.push_back(cd(-1.0, 0.0));
  const int m1 = m + 1;
  double best_err = 1e300, best_a0 = 0.0;
  std::vector<cd> best_reps, best_alpha;
  for (int sweep = 0; sweep < 80; ++sweep) {
    double vn = 0.0;
    for (int i = 0; i < N; ++i) vn += w[i];
    vn = std::sqrt(vn);
    for (int i = 0; i < N; ++i) v0[i] = std::sqrt(w[i]) / vn;
    Mat V, Kp, Hp;
    if (!rational_arnoldi(x, v0, poles, V, Kp, Hp)) {
      msg = "rational Arnoldi breakdown";
      if (best_reps.empty()) return TEM_EBREAKDOWN;
      break;
    }
    // (I - V V^*) F V with F = diag(exp(-x))
    Mat L(N, m1);
    for (int j = 0; j < m1; ++j)
      for (int i = 0; i < N; ++i) L(i, j) = y[i] * V(i, j);
    Mat G(m1, m1);
    for (int j = 0; j < m1; ++j)
      for (int l = 0; l < m1; ++l) {
        cd d(0.0, 0.0);
        for (int i = 0; i < N; ++i) d += std::conj(V(i, l)) * L(i, j);
        G(l, j) = d;
      }
    for (int j = 0; j < m1; ++j)
      for (int i = 0; i < N; ++i) {
        cd s = L(i, j);
        for (int l = 0; l < m1; ++l) s -= V(i, l) * G(l, j);
        L(i, j) = s;
      }
    const std::vector<cd> c = smallest_right_singular(householder_r(L));
    std::vector<cd> z;
    if (!relocated_poles(Hp, Kp, c, z)) {
      msg = "pole relocation failed (singular pencil or no QR convergence)";
      if (best_reps.empty()) return TEM_EBREAKDOWN;
      break;
    }
    poles = symmetrize(z, poles);
    const std::vector<cd> reps = representatives(poles);
    double a0;
    std::vector<cd> alpha;
    fit_with_constant(reps, x, y, w, a0, alpha);
    const double e = single_error(reps, alpha, a0, 4000);
    if (std::isfinite(e) && e < best_err) {
      best_err = e;
      best_reps = reps;
      best_alpha = alpha;
      best_a0 = a0;
    }
    if (sweep + 1 >= 5) {  // Lawson step
      double wmax = 0.0;
      for (int i = 0; i < N; ++i) {
        const double ei = std::abs(y[i] - eval_single(reps, alpha, a0, x[i]));
        w[i] *= std::sqrt(ei);
        wmax = std::max(wmax, w[i]);
      }
      if (!(wmax > 0.0) || !std::isfinite(wmax)) break;
      for (int i = 0; i < N; ++i) w[i] = std::max(w[i] / wmax, 1e-300);
    }
  }
  if (best_reps.empty()) {
    msg = "no finite single-time fit";
    return TEM_EBREAKDOWN;
  }
  out.xi = best_reps;
  out.a.resize(best_reps.size());
  for (size_t j = 0; j < best_reps.size(); ++j) out.a[j] = (best_reps[j].imag() > 0 ? 2.0 : 1.0) * best_alpha[j];
  out.a0 = best_a0;
  out.err = single_error(best_reps, best_alpha, best_a0, 200000);
  return TEM_OK;
}

}  // namespace tem
