// Spectra from dipole series on the GPU (td_spectrum, td_transient_absorption
// in tddftb.h): the polarizability of a kicked run (Sec. 2.2, Eqs. 17-18),
// the effective polarizability of pump-probe runs and the transient
// absorption built from it (Sec. 5.1), with the delay-axis Gaussian filter
// and the absorption change against the end of the pump (Sec. 5.2).
//
// The damped Fourier sums of all series at all frequencies are one dense
// product: D [series x samples] (damped, referenced, scaled differences)
// times B [samples x (cos | sin)] on the FP64 matrix cores (dgemm). The
// delay-axis filter is the circulant matrix of the Gaussian transfer
// function applied as a second product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/tddftb.h"
#include "common.hpp"
#include "ctx.hpp"

using td::round_up;
using tdi::Fail;
using tdi::guarded;
using tdi::set_err;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kLightAu = 137.035999084;   // speed of light, atomic units

struct SpecRun {
  std::string err;
  hipStream_t stream = nullptr;
  std::vector<void*> bufs;
  ~SpecRun() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : bufs) (void)hipFree(p);
    if (stream) (void)hipStreamDestroy(stream);
  }
  double* alloc(size_t count) {
    void* p = nullptr;
    HIPCHK(this, hipMalloc(&p, sizeof(double) * std::max<size_t>(count, 1)));
    bufs.push_back(p);
    HIPCHK(this, hipMemsetAsync(p, 0, sizeof(double) * std::max<size_t>(count, 1), stream));
    return (double*)p;
  }
};

__global__ void k_series(const double* __restrict__ mu, const double* __restrict__ ref,
                         const double* __restrict__ e0, int J, int T, int Tp, double dt,
                         double tau, double* __restrict__ D) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)J * T) return;
  const int j = (int)(idx / T), n = (int)(idx % T);
  const double r = ref ? ref[idx] : mu[(size_t)j * T];
  const double damp = tau > 0.0 ? exp(-(n * dt) / tau) : 1.0;
  D[(size_t)j * Tp + n] = (mu[idx] - r) * damp * dt / e0[j];
}

// B[n][w] = cos(omega_w t_n), B[n][Wp + w] = sin(omega_w t_n).
__global__ void k_basis(const double* __restrict__ omega, int W, int Wp, int T, double dt,
                        double* __restrict__ B) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)T * W) return;
  const int n = (int)(idx / W), w = (int)(idx % W);
  double s, c;
  sincos(omega[w] * (n * dt), &s, &c);
  B[(size_t)n * 2 * Wp + w] = c;
  B[(size_t)n * 2 * Wp + Wp + w] = s;
}

__global__ void k_alpha_out(const double* __restrict__ C, int Wp, int J, int W,
                            const double* __restrict__ omega, double* __restrict__ are,
                            double* __restrict__ aim, double* __restrict__ sig) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)J * W) return;
  const int j = (int)(idx / W), w = (int)(idx % W);
  const double re = C[(size_t)j * 2 * Wp + w], im = C[(size_t)j * 2 * Wp + Wp + w];
  are[idx] = re;
  aim[idx] = im;
  sig[idx] = 4.0 * kPi * omega[w] / kLightAu * im;
}

// sigma[d][w] = 4 pi omega / c * mean_a Im alpha[d * n_avg + a][w], into S [Dp x Wq].
__global__ void k_ta_sigma(const double* __restrict__ C, int Wp, int n_delay, int n_avg, int W,
                           const double* __restrict__ omega, double* __restrict__ S, int Wq) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n_delay * W) return;
  const int d = (int)(idx / W), w = (int)(idx % W);
  double acc = 0.0;
  for (int a = 0; a < n_avg; ++a) acc += C[((size_t)d * n_avg + a) * 2 * Wp + Wp + w];
  S[(size_t)d * Wq + w] = 4.0 * kPi * omega[w] / kLightAu * (acc / n_avg);
}

// Circulant matrix of the periodic Gaussian low-pass over N delays:
// M[a][b] = c[(a - b) mod N], c[m] = 1/N sum_k g_k cos(2 pi k m / N),
// g_k = exp(-nu_k^2 / (2 width^2)), nu_k = k / (N step) folded to |k| <= N/2.
__global__ void k_circulant(int N, int Dp, double step, double width, double* __restrict__ M) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)N * N) return;
  const int a = (int)(idx / N), b = (int)(idx % N);
  const int m = ((a - b) % N + N) % N;
  double acc = 0.0;
  for (int k = 0; k < N; ++k) {
    const int kk = k <= N / 2 ? k : k - N;
    const double nu = kk / (N * step);
    const double g = exp(-nu * nu / (2.0 * width * width));
    acc += g * cos(2.0 * kPi * (double)(((long long)k * m) % N) / N);
  }
  M[(size_t)a * Dp + b] = acc / N;
}

__global__ void k_take(const double* __restrict__ X, int ldx, int n_delay, int W, int ref_row,
                       double* __restrict__ out) {
  const size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (size_t)n_delay * W) return;
  const int d = (int)(idx / W), w = (int)(idx % W);
  const double base = ref_row >= 0 ? X[(size_t)ref_row * ldx + w] : 0.0;
  out[idx] = X[(size_t)d * ldx + w] - base;
}

unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Damped transforms of J series of T samples at W frequencies: C [Jp x 2Wp]
// on the device (Re in columns [0, Wp), Im in [Wp, 2Wp)).
double* transforms(SpecRun* r, int J, int T, const double* mu, const double* ref,
                   const double* e0, double dt, double tau, int W, const double* omega,
                   double** omega_d, int* Wp_out) {
  REQUIRE(r, J > 0 && T >= 2 && W > 0, TD_EINVAL, "need series, >= 2 samples and frequencies");
  REQUIRE(r, mu && e0 && omega, TD_EINVAL, "null input");
  REQUIRE(r, dt > 0 && std::isfinite(dt) && std::isfinite(tau), TD_EINVAL, "invalid dt or tau");
  const size_t JT = (size_t)J * T;
  REQUIRE(r, finite_all(mu, JT) && (!ref || finite_all(ref, JT)) && finite_all(omega, W) &&
                 finite_all(e0, J),
          TD_EINVAL, "non-finite input");
  for (int j = 0; j < J; ++j) REQUIRE(r, e0[j] != 0.0, TD_EINVAL, "kick strength must be non-zero");
  const int Jp = round_up(J, td::kGemmTile), Tp = round_up(T, 16), Wp = round_up(W, 64);
  REQUIRE(r, (double)Jp * Tp + (double)Tp * 2 * Wp + (double)Jp * 2 * Wp < 4.0e9, TD_EINVAL,
          "spectrum too large for one call");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  REQUIRE(r, e == hipSuccess && ndev > 0, TD_EHIP, "no HIP device available");
  HIPCHK(r, hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking));
  double* mu_d = r->alloc(JT);
  double* ref_d = ref ? r->alloc(JT) : nullptr;
  double* e0_d = r->alloc(J);
  double* om_d = r->alloc(W);
  HIPCHK(r, hipMemcpyAsync(mu_d, mu, sizeof(double) * JT, hipMemcpyHostToDevice, r->stream));
  if (ref)
    HIPCHK(r, hipMemcpyAsync(ref_d, ref, sizeof(double) * JT, hipMemcpyHostToDevice, r->stream));
  HIPCHK(r, hipMemcpyAsync(e0_d, e0, sizeof(double) * J, hipMemcpyHostToDevice, r->stream));
  HIPCHK(r, hipMemcpyAsync(om_d, omega, sizeof(double) * W, hipMemcpyHostToDevice, r->stream));
  double* D = r->alloc((size_t)Jp * Tp);
  double* B = r->alloc((size_t)Tp * 2 * Wp);
  double* C = r->alloc((size_t)Jp * 2 * Wp);
  hipLaunchKernelGGL(k_series, dim3(blocks(JT)), dim3(256), 0, r->stream, mu_d, ref_d, e0_d, J, T,
                     Tp, dt, tau, D);
  HIPCHK(r, hipGetLastError());
  hipLaunchKernelGGL(k_basis, dim3(blocks((size_t)T * W)), dim3(256), 0, r->stream, om_d, W, Wp,
                     T, dt, B);
  HIPCHK(r, hipGetLastError());
  HIPCHK(r, td::dgemm(r->stream, 0, Jp, 2 * Wp, Tp, 1.0, D, Tp, B, 2 * Wp, 0.0, nullptr, 0, C,
                      2 * Wp));
  *omega_d = om_d;
  *Wp_out = Wp;
  return C;
}

}  // namespace

extern "C" {

td_status td_spectrum(int32_t n_series, int32_t n_t, const double* mu, const double* ref,
                      const double* e0, double dt, double tau, int32_t n_omega,
                      const double* omega, double* alpha_re, double* alpha_im, double* sigma,
                      char* err, int32_t errlen) {
  SpecRun run;
  SpecRun* r = &run;
  const td_status st = guarded(r, [&] {
    REQUIRE(r, alpha_re && alpha_im && sigma, TD_EINVAL, "null output");
    double* om_d = nullptr;
    int Wp = 0;
    double* C = transforms(r, n_series, n_t, mu, ref, e0, dt, tau, n_omega, omega, &om_d, &Wp);
    const size_t JW = (size_t)n_series * n_omega;
    double* out = r->alloc(3 * JW);
    hipLaunchKernelGGL(k_alpha_out, dim3(blocks(JW)), dim3(256), 0, r->stream, C, Wp, n_series,
                       n_omega, om_d, out, out + JW, out + 2 * JW);
    HIPCHK(r, hipGetLastError());
    HIPCHK(r, hipMemcpyAsync(alpha_re, out, sizeof(double) * JW, hipMemcpyDeviceToHost, r->stream));
    HIPCHK(r, hipMemcpyAsync(alpha_im, out + JW, sizeof(double) * JW, hipMemcpyDeviceToHost,
                             r->stream));
    HIPCHK(r, hipMemcpyAsync(sigma, out + 2 * JW, sizeof(double) * JW, hipMemcpyDeviceToHost,
                             r->stream));
    HIPCHK(r, hipStreamSynchronize(r->stream));
  });
  set_err(err, errlen, st == TD_OK ? "" : run.err);
  return st;
}

td_status td_transient_absorption(int32_t n_delay, int32_t n_avg, int32_t n_t, const double* mu,
                                  const double* ref, const double* e0, double dt, double tau,
                                  int32_t n_omega, const double* omega, int32_t ref_delay,
                                  double delay_step, double filter_width, double* out,
                                  char* err, int32_t errlen) {
  SpecRun run;
  SpecRun* r = &run;
  const td_status st = guarded(r, [&] {
    REQUIRE(r, out && ref, TD_EINVAL, "null output or pump-only reference");
    REQUIRE(r, n_delay > 0 && n_avg > 0 && (int64_t)n_delay * n_avg < (1 << 30), TD_EINVAL,
            "need delays and series per delay");
    REQUIRE(r, ref_delay < n_delay, TD_EINVAL, "ref_delay out of range");
    REQUIRE(r, std::isfinite(filter_width) && (filter_width <= 0 || (delay_step > 0 && std::isfinite(delay_step))),
            TD_EINVAL, "filter needs a positive delay step");
    double* om_d = nullptr;
    int Wp = 0;
    const int J = n_delay * n_avg;
    double* C = transforms(r, J, n_t, mu, ref, e0, dt, tau, n_omega, omega, &om_d, &Wp);
    const int Dp = round_up(n_delay, td::kGemmTile), Wq = round_up(n_omega, td::kGemmTile);
    double* S = r->alloc((size_t)Dp * Wq);
    const size_t DW = (size_t)n_delay * n_omega;
    hipLaunchKernelGGL(k_ta_sigma, dim3(blocks(DW)), dim3(256), 0, r->stream, C, Wp, n_delay,
                       n_avg, n_omega, om_d, S, Wq);
    HIPCHK(r, hipGetLastError());
    double* X = S;
    if (filter_width > 0) {
      double* M = r->alloc((size_t)Dp * Dp);
      double* F = r->alloc((size_t)Dp * Wq);
      hipLaunchKernelGGL(k_circulant, dim3(blocks((size_t)n_delay * n_delay)), dim3(256), 0,
                         r->stream, n_delay, Dp, delay_step, filter_width, M);
      HIPCHK(r, hipGetLastError());
      HIPCHK(r, td::dgemm(r->stream, 0, Dp, Wq, Dp, 1.0, M, Dp, S, Wq, 0.0, nullptr, 0, F, Wq));
      X = F;
    }
    double* o = r->alloc(DW);
    hipLaunchKernelGGL(k_take, dim3(blocks(DW)), dim3(256), 0, r->stream, X, Wq, n_delay, n_omega,
                       ref_delay, o);
    HIPCHK(r, hipGetLastError());
    HIPCHK(r, hipMemcpyAsync(out, o, sizeof(double) * DW, hipMemcpyDeviceToHost, r->stream));
    HIPCHK(r, hipStreamSynchronize(r->stream));
  });
  set_err(err, errlen, st == TD_OK ? "" : run.err);
  return st;
}

}  // extern "C"
