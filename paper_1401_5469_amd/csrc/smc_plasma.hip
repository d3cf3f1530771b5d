// smc_plasma.hip -- plasma state (Kerzendorf & Sim 2014, section 2.3) and
// Sobolev optical depths (section 2.5) on the device.
//
// Two launches per update:
//   plasma_state_kernel  one workgroup per shell: partition functions (one
//                        wavefront per ion, lanes over its levels), the log
//                        ionization ratios, n_e from charge conservation
//                        (one wavefront, lanes over elements, safeguarded
//                        Newton in ln n_e), ion densities and level
//                        populations.  Latency-bound and small: S workgroups
//                        of a few microseconds each.
//   plasma_tau_kernel    one lane per line, looping over shells: two
//                        population gathers (L2-resident, S * n_levels
//                        doubles) and one coalesced 8-byte store per
//                        (shell, line).  HBM-bound on the tau_S stores.
// plasma_lines_kernel runs once at load and folds the oscillator strength,
// the wavelength and t_exp into one coefficient per line.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/smc.h"
#include "smc_internal.h"

namespace smc {
namespace {

// CGS, CODATA 2018
constexpr double kC = 2.99792458e10;
constexpr double kH = 6.62607015e-27;
constexpr double kKB = 1.380649e-16;
constexpr double kME = 9.1093837015e-28;
constexpr double kECharge = 1.602176634e-19 * 2.99792458e9;  // statcoulomb
constexpr double kPi = 3.14159265358979323846;
// pi e^2 / (m_e c): the classical line-strength constant [cm^2 s^-1]
constexpr double kLineConst = kPi * (kECharge * kECharge) / (kME * kC);
// the nebular mode takes the electron temperature as 0.9 T_R
constexpr double kTeOverTr = 0.9;
// n_e is searched in [x_max e^-600, x_max], x_max the largest possible
// charge density of the shell
constexpr double kLogNeRange = 600.0;
constexpr int kNewtonMax = 200;

constexpr int kWave = 64;
constexpr int kStateThreads = 256;
constexpr int kTauThreads = 256;

__device__ inline double wave_sum(double v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Boltzmann weight of a level, with the dilution factor on levels that are
// not metastable in dilute-LTE excitation
__device__ inline double level_weight(const DevPlasma& p, int l, double kT, double W,
                                      bool dilute) {
  double b = p.level_g[l] * exp(-p.level_energy[l] / kT);
  if (dilute && !p.level_meta[l]) b = W * b;
  return b;
}

// Charge moments of one element at ln n_e = u: stage j has log weight
// sum_{m<j} (lphi[a+m] - u) relative to stage 0.  Returns the mean charge and
// its variance (minus the derivative of the mean in u).
__device__ inline void element_moments(const double* lphi, int a, int b, double u, double* q,
                                       double* var) {
  double lr = 0.0, m = 0.0;
  for (int i = a; i < b - 1; ++i) {
    lr += lphi[i] - u;
    m = fmax(m, lr);
  }
  double s0 = exp(-m), s1 = 0.0, s2 = 0.0;
  lr = 0.0;
  for (int i = a; i < b - 1; ++i) {
    lr += lphi[i] - u;
    const double w = exp(lr - m);
    const double j = (double)(i - a + 1);
    s0 += w;
    s1 += j * w;
    s2 += j * j * w;
  }
  *q = s1 / s0;
  *var = fmax(s2 / s0 - *q * *q, 0.0);
}

__global__ __launch_bounds__(kStateThreads) void plasma_state_kernel(DevPlasma p) {
  extern __shared__ double sh[];
  double* Z = sh;                     // [n_ions] partition functions
  double* lphi = sh + p.n_ions;       // [n_ions] log ionization ratios (stage j -> j+1)
  double* N = sh + 2 * p.n_ions;      // [n_ions] ion densities
  __shared__ double s_ne;
  const int s = blockIdx.x;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const double T = p.T_R[s], W = p.W[s];
  const double kT = kKB * T;
  const bool dilute = p.excitation == SMC_EXC_DILUTE_LTE;
  const double* dens = p.density + (size_t)s * p.E;

  // step 1: partition functions, one wavefront per ion
  for (int i = wave; i < p.n_ions; i += kStateThreads / kWave) {
    double z = 0.0;
    for (int l = p.ion_level_ptr[i] + lane; l < p.ion_level_ptr[i + 1]; l += kWave)
      z += level_weight(p, l, kT, W, dilute);
    z = wave_sum(z);
    if (lane == 0) Z[i] = z;
  }
  __syncthreads();

  // step 2: log of N_{j+1} n_e / N_j (Saha, or the nebular form)
  const double log_thermal = 1.5 * log(2.0 * kPi * kME * kT / (kH * kH));
  for (int e = threadIdx.x; e < p.E; e += kStateThreads) {
    const int a = p.elem_ion_ptr[e], b = p.elem_ion_ptr[e + 1];
    for (int i = a; i < b - 1; ++i) {
      double l = log(2.0) + log(Z[i + 1]) - log(Z[i]) + log_thermal - p.ion_chi[i] / kT;
      if (p.ionization == SMC_ION_NEBULAR) {
        const double z = p.ion_zeta[i];
        l = l + log(W * (p.delta * z + W * (1.0 - z))) + 0.5 * log(kTeOverTr);
      }
      lphi[i] = l;
    }
    lphi[b - 1] = -INFINITY;
  }
  __syncthreads();

  // step 3: n_e from charge conservation; g(u) = sum_e N_e q_e(u) - e^u is
  // strictly decreasing in u = ln n_e, so Newton steps are kept inside a
  // bracket that every evaluation narrows
  if (wave == 0) {
    double xmax = 0.0;
    for (int e = lane; e < p.E; e += kWave)
      xmax += dens[e] * (double)(p.elem_ion_ptr[e + 1] - p.elem_ion_ptr[e] - 1);
    xmax = wave_sum(xmax);
    double x = 0.0;
    if (xmax > 0.0) {
      double hi = log(xmax), lo = hi - kLogNeRange, u = hi;
      for (int it = 0; it < kNewtonMax; ++it) {
        double sq = 0.0, sv = 0.0;
        for (int e = lane; e < p.E; e += kWave) {
          const double Ne = dens[e];
          if (Ne > 0.0) {
            double q, var;
            element_moments(lphi, p.elem_ion_ptr[e], p.elem_ion_ptr[e + 1], u, &q, &var);
            sq += Ne * q;
            sv += Ne * var;
          }
        }
        sq = wave_sum(sq);
        sv = wave_sum(sv);
        const double xu = exp(u);
        const double g = sq - xu;
        if (g > 0.0) lo = u;
        else hi = u;
        double un = u - g / (-sv - xu);
        if (!(un > lo && un < hi)) un = 0.5 * (lo + hi);
        const bool done = fabs(un - u) <= 1e-15 * fmax(1.0, fabs(u)) || !(hi > lo);
        u = un;
        if (done) break;
      }
      x = exp(u);
    }
    // ion densities at that n_e
    const double lx = x > 0.0 ? log(x) : 0.0;
    for (int e = lane; e < p.E; e += kWave) {
      const int a = p.elem_ion_ptr[e], b = p.elem_ion_ptr[e + 1];
      const double Ne = dens[e];
      if (x > 0.0) {
        double lr = 0.0, m = 0.0;
        for (int i = a; i < b - 1; ++i) {
          lr += lphi[i] - lx;
          m = fmax(m, lr);
        }
        double s0 = exp(-m);
        lr = 0.0;
        for (int i = a; i < b - 1; ++i) {
          lr += lphi[i] - lx;
          s0 += exp(lr - m);
        }
        N[a] = Ne * (exp(-m) / s0);
        lr = 0.0;
        for (int i = a; i < b - 1; ++i) {
          lr += lphi[i] - lx;
          N[i + 1] = Ne * (exp(lr - m) / s0);
        }
      } else {
        // no charge is possible: every element sits in its only stage
        for (int i = a; i < b; ++i) N[i] = i == a ? Ne : 0.0;
      }
    }
    if (lane == 0) s_ne = x;
  }
  __syncthreads();

  for (int i = threadIdx.x; i < p.n_ions; i += kStateThreads) {
    p.partition[(size_t)s * p.n_ions + i] = Z[i];
    p.ion_density[(size_t)s * p.n_ions + i] = N[i];
  }
  if (threadIdx.x == 0) {
    p.n_e[s] = s_ne;
    if (s == 0) p.clamped[0] = 0ull;  // the depth kernel runs after this one
  }
  // step 4: level populations
  double* pop = p.level_pop + (size_t)s * p.n_levels;
  for (int l = threadIdx.x; l < p.n_levels; l += kStateThreads) {
    const int i = p.level_ion[l];
    pop[l] = N[i] / Z[i] * level_weight(p, l, kT, W, dilute);
  }
}

// step 5: Sobolev depths, one lane per line
__global__ __launch_bounds__(kTauThreads) void plasma_tau_kernel(DevPlasma p) {
  const int k = blockIdx.x * kTauThreads + threadIdx.x;
  unsigned long long neg = 0;
  if (k < p.L) {
    const PlasmaLine ln = p.lines[k];
    const double* pop = p.level_pop;
    double* tau = p.tau + k;
    for (int s = 0; s < p.S; ++s) {
      const double nl = pop[ln.lower], nu = pop[ln.upper];
      const double stim = nl > 0.0 ? 1.0 - ln.g_l * nu / (ln.g_u * nl) : 0.0;
      double t = ln.coef * nl * stim;
      if (t < 0.0) {
        t = 0.0;
        ++neg;
      }
      *tau = t;
      pop += p.n_levels;
      tau += p.Lp;
    }
  }
  neg = wave_sum_u64(neg);
  if ((threadIdx.x % kWave) == 0 && neg) atomicAdd(p.clamped, neg);
}

__global__ void plasma_lines_kernel(DevPlasma p) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= p.L) return;
  p.lines[k].coef = kLineConst * p.line_f[k] * (kC / p.line_nu[k]) * p.t_exp;
}

}  // namespace

hipError_t launch_plasma_lines(const DevPlasma& p, hipStream_t s) {
  if (p.L == 0) return hipSuccess;
  hipLaunchKernelGGL(plasma_lines_kernel, dim3((p.L + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_plasma_update(const DevPlasma& p, hipStream_t s) {
  const size_t lds = 3 * (size_t)p.n_ions * sizeof(double);
  hipLaunchKernelGGL(plasma_state_kernel, dim3(p.S), dim3(kStateThreads), lds, s, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || p.L == 0) return e;
  hipLaunchKernelGGL(plasma_tau_kernel, dim3((p.L + kTauThreads - 1) / kTauThreads),
                     dim3(kTauThreads), 0, s, p);
  return hipGetLastError();
}

}  // namespace smc
