// Batch autoregressive sampling (BAS) on the GPU.
//
// The N_s samples are a tree of unique prefixes with multiplicities. For orbital k:
// the FP64 ansatz gives every prefix its number-conserving conditional over the four
// occupations of orbital k; every prefix splits its weight w among the occupations by one
// multinomial draw (a chain of binomials, one thread per prefix), so a step costs the same
// for any N_s; children with no draws are pruned and the rest listed in (prefix, state)
// order by an exclusive scan. The uniforms come from Philox4x32-10 at counter
// (attempt, prefix, k, state) and key (seed), so the tree does not depend on scheduling.
// The prefix counts live in device memory: no step waits for the host.
#include <cmath>

#include "elocal_internal.hpp"
#include "kernels.hpp"

namespace elocal {

// ----------------------------------------------------------------------------- Philox4x32-10
// Salmon et al., SC 2011: 10 rounds of (hi, lo) = M * c on words 0 and 2, with the Weyl
// key schedule (0x9E3779B9, 0xBB67AE85).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// The two uniforms in [0, 1) of attempt t of the binomial of state st of prefix i at
// orbital k: the 53 high bits of words (0, 1) and of words (2, 3).
struct UniformStream {
  uint32_t i, k, st;
  uint64_t seed;
  __device__ __forceinline__ void pair(uint32_t t, double& u1, double& u2) const {
    uint32_t c[4] = {t, i, k, st};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    u1 = (double)((((uint64_t)c[0] << 32) | c[1]) >> 11) * 0x1.0p-53;
    u2 = (double)((((uint64_t)c[2] << 32) | c[3]) >> 11) * 0x1.0p-53;
  }
};

// The binomial arithmetic below is written as plain FP64 operations in a fixed order, not
// contracted into fused multiply-adds, so its rounding is that of the same expressions
// evaluated one operation at a time.
#pragma clang fp contract(off)

// Stirling-series correction f_c(k) = ln k! - (k + 1/2) ln(k + 1) + (k + 1) - ln(2 pi)/2
// of the BTRD acceptance test (Hormann 1993): from its definition below 10, else from the
// series 1/12 - 1/360 (k+1)^-2 + 1/1260 (k+1)^-4, over (k + 1).
__device__ double stirling_fc(double k) {
  if (k < 10.0) return lgamma(k + 1.0) - (k + 0.5) * log(k + 1.0) + (k + 1.0) - 0.5 * log(2.0 * M_PI);
  const double kk = 1.0 / ((k + 1.0) * (k + 1.0));
  return (1.0 / 12.0 - (1.0 / 360.0 - 1.0 / 1260.0 * kk) * kk) / (k + 1.0);
}

// Binomial(n, p) with p <= 1/2: inversion from K = 0 when n p < 10 (an attempt that runs
// past the last representable pmf term is retried with the next uniforms), otherwise the
// transformed rejection with decomposition BTRD (W. Hormann, "The generation of binomial
// random variates", J. Stat. Comput. Simul. 46, 1993). n < 2^53.
__device__ int64_t binomial_small_p(int64_t n, double p, const UniformStream& rs) {
  const double nf = (double)n;
  uint32_t t = 0;
  if (nf * p < 10.0) {
    const double s = p / (1.0 - p), a = (nf + 1.0) * s, f0 = exp(nf * log1p(-p));
    for (;;) {
      double u, unused;
      rs.pair(t++, u, unused);
      double f = f0;
      int64_t kk = 0;
      bool ran_out = false;
      while (u > f) {
        u -= f;
        ++kk;
        f *= a / (double)kk - s;
        if (f <= 0.0 || kk > n) { ran_out = true; break; }
      }
      if (!ran_out || (u <= f && kk <= n)) return kk;
    }
  }
  const double m = floor((nf + 1.0) * p);
  const double r = p / (1.0 - p), nr = (nf + 1.0) * r, npq = nf * p * (1.0 - p), spq = sqrt(npq);
  const double b = 1.15 + 2.53 * spq, a = -0.0873 + 0.0248 * b + 0.01 * p, c = nf * p + 0.5;
  const double alpha = (2.83 + 5.1 / b) * spq, vr = 0.92 - 4.2 / b, urvr = 0.86 * vr;
  for (;;) {
    double v, u2, u;
    rs.pair(t++, v, u2);
    if (v <= urvr) {
      u = v / vr - 0.43;
      const double kf = floor((2.0 * a / (0.5 - fabs(u)) + b) * u + c);
      if (kf >= 0.0 && kf <= nf) return (int64_t)kf;
      continue;
    }
    if (v >= vr) {
      u = u2 - 0.5;
    } else {
      u = v / vr - 0.93;
      u = (u > 0.0 ? 0.5 : -0.5) - u;
      v = u2 * vr;
    }
    const double us = 0.5 - fabs(u);
    const double kf = floor((2.0 * a / us + b) * u + c);
    if (kf < 0.0 || kf > nf) continue;
    v = v * alpha / (a / (us * us) + b);
    const double km = fabs(kf - m);
    if (km <= 15.0) {
      double f = 1.0;
      if (m < kf) {
        for (double i = m + 1.0; i <= kf; i += 1.0) f *= nr / i - r;
      } else if (m > kf) {
        for (double i = kf + 1.0; i <= m; i += 1.0) v *= nr / i - r;
      }
      if (v <= f) return (int64_t)kf;
      continue;
    }
    v = log(v);
    const double rho = (km / npq) * (((km / 3.0 + 0.625) * km + 1.0 / 6.0) / npq + 0.5);
    const double tt = -km * km / (2.0 * npq);
    if (v < tt - rho) return (int64_t)kf;
    if (v > tt + rho) continue;
    const double nm = nf - m + 1.0;
    const double h = (m + 0.5) * log((m + 1.0) / (r * nm)) + stirling_fc(m) + stirling_fc(nf - m);
    const double nk = nf - kf + 1.0;
    if (v <= h + (nf + 1.0) * log(nm / nk) + (kf + 0.5) * log(nk * r / (kf + 1.0)) - stirling_fc(kf) -
                  stirling_fc(nf - kf))
      return (int64_t)kf;
  }
}

__device__ int64_t binomial(int64_t n, double p, const UniformStream& rs) {
  if (n <= 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  if (p > 0.5) return n - binomial_small_p(n, 1.0 - p, rs);
  return binomial_small_p(n, p, rs);
}

#pragma clang fp contract(on)

// ----------------------------------------------------------------------------- kernels
// Multinomial split of every prefix's weight over the four occupations of orbital k, one
// thread per prefix: the feasible states (probability > 0) in ascending order take
// binomials of what is left with probability p_s / (sum of the remaining p, in ascending
// order); the last feasible state takes the rest. counts[i][s].
#pragma clang fp contract(off)
__global__ void __launch_bounds__(256) k_bas_split(const double* __restrict__ probs, const int64_t* __restrict__ w,
                                                   const int64_t* __restrict__ ucur, int64_t cap, int k,
                                                   uint64_t seed, int64_t* __restrict__ counts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= min(*ucur, cap)) return;
  double p[4];
  int last = -1;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    p[q] = probs[4 * i + q];
    if (p[q] > 0.0) last = q;
  }
  int64_t left = w[i];
  int64_t c[4] = {0, 0, 0, 0};
  UniformStream rs{(uint32_t)i, (uint32_t)k, 0u, seed};
  for (int q = 0; q < last; ++q) {
    if (!(p[q] > 0.0)) continue;
    double rem = 0.0;
    for (int q2 = q; q2 < 4; ++q2)
      if (p[q2] > 0.0) rem = rem + p[q2];
    rs.st = (uint32_t)q;
    const int64_t cq = binomial(left, fmin(1.0, p[q] / rem), rs);
    c[q] = cq;
    left -= cq;
  }
  if (last >= 0) c[last] = left;
#pragma unroll
  for (int q = 0; q < 4; ++q) counts[4 * i + q] = c[q];
}
#pragma clang fp contract(on)

// Number of surviving children per prefix, and their exclusive scan (blocks of 1024,
// then the block totals, then the block offsets added).
__global__ void __launch_bounds__(1024) k_bas_scan_blocks(const int64_t* __restrict__ counts,
                                                          const int64_t* __restrict__ ucur, int64_t cap,
                                                          int64_t* __restrict__ off, int64_t* __restrict__ btot) {
  __shared__ int64_t s[1024];
  const int64_t U = min(*ucur, cap);
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  int64_t v = 0;
  if (i < U)
    for (int q = 0; q < 4; ++q) v += counts[4 * i + q] > 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t t = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < U) off[i] = s[threadIdx.x] - v;   // exclusive within the block
  if (threadIdx.x == 1023) btot[blockIdx.x] = s[1023];
}

__global__ void __launch_bounds__(1024) k_bas_scan_totals(int64_t* __restrict__ btot, int64_t nblk,
                                                          int64_t* __restrict__ total, int64_t cap,
                                                          int64_t* __restrict__ overflow) {
  __shared__ int64_t s[1024];
  int64_t carry = 0;
  for (int64_t base = 0; base < nblk; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nblk ? btot[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int64_t t = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < nblk) btot[i] = carry + s[threadIdx.x] - v;   // exclusive block offsets
    carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *total = carry;
    if (overflow && carry > cap) *overflow = 1;
  }
}

template <int NW>
__global__ void k_bas_emit(const uint64_t* __restrict__ pre, const int64_t* __restrict__ counts,
                           const int64_t* __restrict__ ucur, int k, const int64_t* __restrict__ off,
                           const int64_t* __restrict__ btot, uint64_t* __restrict__ child, int64_t* __restrict__ cw,
                           int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= min(*ucur, cap)) return;
  int64_t o = off[i] + btot[i / 1024];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int64_t c = counts[4 * i + s];
    if (c <= 0) continue;
    if (o < cap) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        uint64_t v = pre[i * NW + w];
        const int ka = 2 * k, kb = 2 * k + 1;
        if ((s & 1) && (ka >> 6) == w) v |= 1ull << (ka & 63);
        if ((s & 2) && (kb >> 6) == w) v |= 1ull << (kb & 63);
        child[o * NW + w] = v;
      }
      cw[o] = c;
    }
    ++o;
  }
}

__global__ void k_bas_root(uint64_t* pre, int64_t* w, int W, int64_t n_samples, int64_t* u0, int64_t* overflow) {
  if (threadIdx.x < (unsigned)W) pre[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) {
    w[0] = n_samples;
    *u0 = 1;
    *overflow = 0;
  }
}

// ----------------------------------------------------------------------------- launchers
hipError_t launch_bas_root(uint64_t* pre, int64_t* w, int W, int64_t n_samples, int64_t* u0, int64_t* overflow,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_bas_root, dim3(1), dim3(64), 0, st, pre, w, W, n_samples, u0, overflow);
  return hipGetLastError();
}

hipError_t launch_bas_step(const SysDev& S, const MadeDev& M, int hmax, const uint64_t* pre, const int64_t* w,
                           const int64_t* ucur, int64_t* unext, int64_t* overflow, int k, uint64_t seed, double* probs,
                           int64_t* counts, int64_t* off, int64_t* btot, uint64_t* child, int64_t* cw, int64_t cap,
                           hipStream_t st) {
  if (cap <= 0) return hipErrorInvalidValue;
  hipError_t e = launch_bas_probs(S, M, hmax, pre, ucur, cap, k, probs, st);
  if (e != hipSuccess) return e;
  const int64_t nblk = (cap + 1023) / 1024;
  const unsigned tb = (unsigned)((cap + 255) / 256);
  hipLaunchKernelGGL(k_bas_split, dim3(tb), dim3(256), 0, st, probs, w, ucur, cap, k, seed, counts);
  hipLaunchKernelGGL(k_bas_scan_blocks, dim3((unsigned)nblk), dim3(1024), 0, st, counts, ucur, cap, off, btot);
  hipLaunchKernelGGL(k_bas_scan_totals, dim3(1), dim3(1024), 0, st, btot, nblk, unext, cap, overflow);
  if (S.W == 1)
    hipLaunchKernelGGL(k_bas_emit<1>, dim3(tb), dim3(256), 0, st, pre, counts, ucur, k, off, btot, child, cw, cap);
  else
    hipLaunchKernelGGL(k_bas_emit<2>, dim3(tb), dim3(256), 0, st, pre, counts, ucur, k, off, btot, child, cw, cap);
  return hipGetLastError();
}

}  // namespace elocal
