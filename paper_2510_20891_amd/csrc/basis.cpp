// build_basis: centred SVD basis of training frequency tracks (Sec. II C,
// Eqs. (9)-(10)) and the uniform coefficient box from symmetric 3-sigma
// quantiles of the training projections.  Host code, FP64, synchronous.
//
// The n_train x n_seg matrix X of centred tracks is reduced by Householder QR
// to its n x n triangular factor R (n = n_seg; skipped when n_train < n_seg),
// and the right singular vectors are obtained by one-sided (Hestenes) Jacobi
// rotations of R's columns, accumulated in V.  Column norms of the rotated
// matrix are the singular values.  This keeps the small singular directions
// accurate (no Gram matrix is formed).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"

namespace {

// In-place Householder QR of the m x n column-major matrix A (m >= n); returns
// the n x n upper-triangular R, column-major.
std::vector<double> householder_r(std::vector<double> &A, int64_t m, int n) {
  std::vector<double> v(m);
  for (int k = 0; k < n; ++k) {
    double *ak = &A[(size_t)k * m];
    double norm2 = 0.0;
    for (int64_t i = k; i < m; ++i) norm2 += ak[i] * ak[i];
    const double norm = std::sqrt(norm2);
    if (norm == 0.0) continue;
    const double alpha = ak[k] > 0 ? -norm : norm;
    for (int64_t i = k; i < m; ++i) v[i] = ak[i];
    v[k] -= alpha;
    double vnorm2 = 0.0;
    for (int64_t i = k; i < m; ++i) vnorm2 += v[i] * v[i];
    if (vnorm2 == 0.0) continue;
    for (int j = k; j < n; ++j) {
      double *aj = &A[(size_t)j * m];
      double d = 0.0;
      for (int64_t i = k; i < m; ++i) d += v[i] * aj[i];
      const double f = 2.0 * d / vnorm2;
      for (int64_t i = k; i < m; ++i) aj[i] -= f * v[i];
    }
  }
  std::vector<double> R((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i <= j; ++i) R[(size_t)j * n + i] = A[(size_t)j * m + i];
  return R;
}

// One-sided Jacobi on the columns of the r x n column-major matrix B; V (n x n,
// column-major) accumulates the rotations so that B_in V = B_out.
void hestenes_jacobi(std::vector<double> &B, int64_t r, int n, std::vector<double> &V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double *bp = &B[(size_t)p * r], *bq = &B[(size_t)q * r];
        double a = 0.0, b = 0.0, g = 0.0;
        for (int64_t i = 0; i < r; ++i) {
          a += bp[i] * bp[i];
          b += bq[i] * bq[i];
          g += bp[i] * bq[i];
        }
        if (g == 0.0 || std::fabs(g) <= tol * std::sqrt(a * b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t);
        const double s = c * t;
        for (int64_t i = 0; i < r; ++i) {
          const double x = bp[i], y = bq[i];
          bp[i] = c * x - s * y;
          bq[i] = s * x + c * y;
        }
        double *vp = &V[(size_t)p * n], *vq = &V[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          const double x = vp[i], y = vq[i];
          vp[i] = c * x - s * y;
          vq[i] = s * x + c * y;
        }
      }
    }
    if (!rotated) break;
  }
}

// Linear-interpolation quantile of sorted data (order statistic at q (n-1)).
double quantile_sorted(const std::vector<double> &v, double q) {
  const size_t n = v.size();
  if (n == 1) return v[0];
  const double h = q * (double)(n - 1);
  const size_t lo = (size_t)std::floor(h);
  const size_t hi = lo + 1 < n ? lo + 1 : lo;
  const double frac = h - (double)lo;
  return v[lo] + (v[hi] - v[lo]) * frac;
}

}  // namespace

extern "C" int build_basis(const double *tracks, int64_t n_train, int32_t n_seg, int32_t K, double *f0, double *U,
                           double *sv, double *box_lo, double *box_hi) {
  using namespace emri;
  clear_error();
  if (!tracks || !f0) return fail(EMRI_EINVAL, "tracks or f0 is NULL");
  if (n_train < 1 || n_seg < 1) return fail(EMRI_EINVAL, "n_train and n_seg must be >= 1");
  if (K < 0 || (int64_t)K > std::min<int64_t>(n_train, n_seg)) return fail(EMRI_EINVAL, "K outside [0, min(n_train, n_seg)]");
  if (K > 0 && (!U || !sv || !box_lo || !box_hi)) return fail(EMRI_EINVAL, "an output array is NULL");
  if (n_train > ((int64_t)1 << 40) / n_seg) return fail(EMRI_ERANGE, "training matrix too large");
  const int n = n_seg;
  const int64_t m = n_train;
  for (int64_t i = 0; i < m * n; ++i)
    if (!std::isfinite(tracks[i])) return fail(EMRI_EINVAL, "training track entry %lld is not finite", (long long)i);

  // f0 = mean track; X = tracks - f0
  std::vector<double> mean(n, 0.0);
  for (int64_t i = 0; i < m; ++i)
    for (int a = 0; a < n; ++a) mean[a] += tracks[i * n + a];
  for (int a = 0; a < n; ++a) mean[a] /= (double)m;
  std::vector<double> X((size_t)(m * n));
  for (int64_t i = 0; i < m; ++i)
    for (int a = 0; a < n; ++a) X[i * n + a] = tracks[i * n + a] - mean[a];
  std::memcpy(f0, mean.data(), sizeof(double) * n);
  if (K == 0) return EMRI_OK;

  // column-major copy of X
  std::vector<double> B((size_t)(m * n));
  for (int64_t i = 0; i < m; ++i)
    for (int a = 0; a < n; ++a) B[(size_t)a * m + i] = X[i * n + a];
  int64_t rows = m;
  if (m >= n) {
    B = householder_r(B, m, n);
    rows = n;
  }
  std::vector<double> V;
  hestenes_jacobi(B, rows, n, V);
  std::vector<double> norms(n);
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < rows; ++i) s += B[(size_t)j * rows + i] * B[(size_t)j * rows + i];
    norms[j] = std::sqrt(s);
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return norms[x] > norms[y]; });

  for (int k = 0; k < K; ++k) {
    const int col = order[k];
    sv[k] = norms[col];
    // sign rule: the largest-magnitude entry (lowest alpha on ties) is positive
    int pivot = 0;
    double best = -1.0;
    for (int a = 0; a < n; ++a) {
      const double v = std::fabs(V[(size_t)col * n + a]);
      if (v > best) { best = v; pivot = a; }
    }
    const double sgn = V[(size_t)col * n + pivot] < 0 ? -1.0 : 1.0;
    for (int a = 0; a < n; ++a) U[(size_t)a * K + k] = sgn * V[(size_t)col * n + a];
  }

  // projections C = X U and their quantile box
  std::vector<double> proj((size_t)m);
  for (int k = 0; k < K; ++k) {
    for (int64_t i = 0; i < m; ++i) {
      double s = 0.0;
      for (int a = 0; a < n; ++a) s += X[i * n + a] * U[(size_t)a * K + k];
      proj[i] = s;
    }
    std::sort(proj.begin(), proj.end());
    box_lo[k] = quantile_sorted(proj, 0.00135);
    box_hi[k] = quantile_sorted(proj, 0.99865);
  }
  return EMRI_OK;
}

namespace emri {

// Pseudo-inverse of the n x K row-major matrix U, written transposed: pt[a*K + k]
// = pinv(U)[k, a].  One-sided Jacobi on U's columns gives U V = B with
// orthogonal columns b_j of norms s_j, so U = B V^T and pinv(U) = V S^-2 B^T;
// directions with s_j <= 1e-15 max s are dropped (rank-deficient U).
void pseudo_inverse_t(const double *U, int n, int K, double *pt) {
  std::vector<double> B((size_t)n * K);
  for (int a = 0; a < n; ++a)
    for (int k = 0; k < K; ++k) B[(size_t)k * n + a] = U[(size_t)a * K + k];
  std::vector<double> V;
  hestenes_jacobi(B, n, K, V);
  std::vector<double> s2(K);
  double smax = 0.0;
  for (int j = 0; j < K; ++j) {
    double q = 0.0;
    for (int a = 0; a < n; ++a) q += B[(size_t)j * n + a] * B[(size_t)j * n + a];
    s2[j] = q;
    smax = std::max(smax, std::sqrt(q));
  }
  std::fill(pt, pt + (size_t)n * K, 0.0);
  for (int j = 0; j < K; ++j) {
    if (!(std::sqrt(s2[j]) > 1e-15 * smax)) continue;
    for (int a = 0; a < n; ++a) {
      const double w = B[(size_t)j * n + a] / s2[j];
      for (int k = 0; k < K; ++k) pt[(size_t)a * K + k] += V[(size_t)j * K + k] * w;
    }
  }
}

}  // namespace emri
