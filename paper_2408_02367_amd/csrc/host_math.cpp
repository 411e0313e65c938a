// Host-side plan mathematics in FP64: kernel parameters, deapodisation,
// piecewise-polynomial kernel fit, FFT radix plans and twiddles.
//
// The NUFFT inside the forward operator (Sec. 2) is read as a Kaiser-Bessel
// gridding NUFFT: width W fine cells, oversampling sigma, shape parameter
// from Beatty, Nishimura and Pauly (2005).  Everything here is computed in
// double precision once per plan and handed to the kernels in float.
#include <cmath>
#include <cstring>
#include <thread>

#include "sdn_internal.h"

namespace sdn {

namespace {
thread_local std::string g_last_error;
}

sdn_status fail(sdn_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

sdn_status hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return SDN_OK;
  return fail(e == hipErrorOutOfMemory ? SDN_E_NOMEM : SDN_E_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

const char *last_error() { return g_last_error.c_str(); }

double kb_beta(int W, double sigma) {
  const double a = (W / sigma) * (sigma - 0.5);
  return M_PI * std::sqrt(a * a - 0.8);
}

// Modified Bessel function of the first kind, order 0, by its power series
// sum_m (x^2/4)^m / (m!)^2 (all terms positive, so no cancellation).
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int m = 1; m < 500; ++m) {
    term *= q / (double(m) * double(m));
    sum += term;
    if (term < 1e-18 * sum) break;
  }
  return sum;
}

// phi(u) = I0(beta sqrt(1 - (2u/W)^2)) on |u| <= W/2, zero outside.
double kb_phi(double u, int W, double beta) {
  const double a = 1.0 - (2.0 * u / W) * (2.0 * u / W);
  if (a < 0.0) return 0.0;
  return bessel_i0(beta * std::sqrt(a));
}

// Continuous Fourier transform of phi at xi cycles per cell:
// W sinh(z) / z with z = sqrt(beta^2 - (pi W xi)^2).
double kb_phi_hat(double xi, int W, double beta) {
  const double z2 = beta * beta - (M_PI * W * xi) * (M_PI * W * xi);
  if (z2 <= 0.0) return NAN;
  const double z = std::sqrt(z2);
  return W * std::sinh(z) / z;
}

bool smooth7(int64_t n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Fine grid: the smallest even 2,3,5,7-smooth length >= max(sigma N, 2W).
int fine_size(int64_t n, double sigma, int W) {
  int64_t m = (int64_t)std::ceil(sigma * (double)n - 1e-9);
  if (m < 2 * W) m = 2 * W;
  if (m % 2) ++m;
  while (!smooth7(m)) m += 2;
  return (int)m;
}

int kernel_ncoef(int W) {
  int n = W + 4;
  return n > kMaxCoef ? kMaxCoef : n;
}

// Fit each of the W kernel pieces g_i(t) = phi(t + W/2 - 1 - i) / I0(beta),
// t in [0,1), by Chebyshev interpolation in z = 2t - 1 at `ncoef` Chebyshev
// points, then expand the Chebyshev series into monomials of z.  Node i of
// a point with fractional offset t lies at distance u = t + W/2 - 1 - i.
void kernel_coefficients(int W, double beta, int ncoef, KerCoef *out) {
  std::memset(out, 0, sizeof(*out));
  const double norm = 1.0 / bessel_i0(beta);
  const int n = ncoef;
  std::vector<double> zk(n), fk(n), a(n), mono(n), tprev(n), tcur(n), tnext(n);
  for (int i = 0; i < W; ++i) {
    for (int q = 0; q < n; ++q) {
      zk[q] = std::cos(M_PI * (q + 0.5) / n);
      const double t = 0.5 * (zk[q] + 1.0);
      fk[q] = kb_phi(t + 0.5 * W - 1.0 - i, W, beta) * norm;
    }
    for (int m = 0; m < n; ++m) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += fk[q] * std::cos(m * M_PI * (q + 0.5) / n);
      a[m] = (m == 0 ? 1.0 : 2.0) * s / n;
    }
    // monomial coefficients of sum_m a_m T_m(z), T_{m+1} = 2 z T_m - T_{m-1}
    std::fill(mono.begin(), mono.end(), 0.0);
    std::fill(tprev.begin(), tprev.end(), 0.0);
    std::fill(tcur.begin(), tcur.end(), 0.0);
    tprev[0] = 1.0;           // T_0
    if (n > 1) tcur[1] = 1.0; // T_1
    mono[0] += a[0];
    for (int m = 1; m < n; ++m) {
      for (int d = 0; d < n; ++d) mono[d] += a[m] * tcur[d];
      std::fill(tnext.begin(), tnext.end(), 0.0);
      for (int d = 0; d + 1 < n; ++d) tnext[d + 1] += 2.0 * tcur[d];
      for (int d = 0; d < n; ++d) tnext[d] -= tprev[d];
      tprev.swap(tcur);
      tcur.swap(tnext);
    }
    for (int d = 0; d < n; ++d) out->c[i][d] = (float)mono[d];
  }
}

// Radix passes for one FFT length: as many radix-8 passes as the power of
// two allows, the leftover two folded into a radix-6 (with a 3) or split as
// 4*4, then the odd radices 3, 5, 7.
RadixPlan radix_plan(int L) {
  RadixPlan rp{};
  rp.L = L;
  int m = L, e2 = 0, e3 = 0, e5 = 0, e7 = 0;
  while (m % 2 == 0) { m /= 2; ++e2; }
  while (m % 3 == 0) { m /= 3; ++e3; }
  while (m % 5 == 0) { m /= 5; ++e5; }
  while (m % 7 == 0) { m /= 7; ++e7; }
  if (m != 1) { rp.n = -1; return rp; }
  std::vector<int> r;
  int n8 = e2 / 3, rem = e2 % 3;
  if (rem == 1) {
    if (e3 > 0) { r.push_back(6); --e3; }
    else if (n8 > 0) { --n8; r.push_back(4); r.push_back(4); }
    else r.push_back(2);
  } else if (rem == 2) {
    r.push_back(4);
  }
  for (int i = 0; i < n8; ++i) r.push_back(8);
  for (int i = 0; i < e7; ++i) r.push_back(7);
  for (int i = 0; i < e5; ++i) r.push_back(5);
  for (int i = 0; i < e3; ++i) r.push_back(3);
  if ((int)r.size() > kMaxRadices) { rp.n = -1; return rp; }
  rp.n = (int)r.size();
  for (int i = 0; i < rp.n; ++i) rp.r[i] = r[i];
  return rp;
}

// 1 / phi_hat(n / nf) for array index q = n + floor(N/2), scaled by I0(beta)
// to match the normalised kernel.
std::vector<float> deapod_inverse(int N, int nf, int W, double beta) {
  std::vector<float> out(N);
  const double i0b = bessel_i0(beta);
  for (int q = 0; q < N; ++q) {
    const double n = q - N / 2;
    out[q] = (float)(i0b / kb_phi_hat(n / nf, W, beta));
  }
  return out;
}

// exp(-2 pi i m / L) for m in [0, L).
std::vector<float> twiddles(int L) {
  std::vector<float> out(2 * (size_t)L);
  for (int m = 0; m < L; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)L;
    out[2 * m] = (float)std::cos(a);
    out[2 * m + 1] = (float)std::sin(a);
  }
  return out;
}

}  // namespace sdn

extern "C" sdn_status sdn_kernel_tables(int W, double sigma, int64_t N, double *beta, int *nf,
                                        int *ncoef, float *coef, float *deapod_inv) {
  using namespace sdn;
  if (W != 4 && W != 6 && W != 8) return fail(SDN_E_UNSUPPORTED, "sdn_kernel_tables: W");
  if (!(sigma >= 1.25 && sigma <= 4.0) || N < 1 || N > 4096 || !beta || !nf || !ncoef || !coef)
    return fail(SDN_E_INVALID, "sdn_kernel_tables: bad argument");
  *beta = kb_beta(W, sigma);
  *nf = fine_size(N, sigma, W);
  *ncoef = kernel_ncoef(W);
  KerCoef kc;
  kernel_coefficients(W, *beta, *ncoef, &kc);
  for (int i = 0; i < kMaxW; ++i)
    for (int d = 0; d < kMaxCoef; ++d) coef[i * kMaxCoef + d] = kc.c[i][d];
  if (deapod_inv) {
    auto t = deapod_inverse((int)N, *nf, W, *beta);
    for (int64_t q = 0; q < N; ++q) deapod_inv[q] = t[q];
  }
  return SDN_OK;
}
