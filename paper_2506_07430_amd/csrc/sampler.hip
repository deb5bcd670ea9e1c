// Batch autoregressive sampling (BAS) on the GPU.
//
// The N_s samples are a tree of unique prefixes with multiplicities. For orbital k:
// the FP64 ansatz gives every prefix its number-conserving conditional over the four
// occupations of orbital k; every prefix splits its weight w by w independent
// categorical draws (uniforms from Philox4x32-10 at counter (draw, prefix, k, 0) and key
// (seed)); children with no draws are pruned and the rest listed in (prefix, state)
// order by an exclusive scan. The draw counts are integer sums, so the tree does not
// depend on scheduling.
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

__device__ __forceinline__ double bas_uniform(uint32_t j, uint32_t i, uint32_t k, uint64_t seed) {
  uint32_t c[4] = {j, i, k, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t bits = (((uint64_t)c[0] << 32) | c[1]) >> 11;
  return (double)bits * 0x1.0p-53;
}

// ----------------------------------------------------------------------------- kernels
// Draw counts of prefix i (gridDim.y blocks per prefix): counts[i][s].
__global__ void __launch_bounds__(256) k_bas_counts(const double* __restrict__ probs, const int64_t* __restrict__ w,
                                                    int k, uint64_t seed, int64_t* __restrict__ counts) {
  __shared__ unsigned long long cnt[4];
  const int64_t i = blockIdx.x;
  if (threadIdx.x < 4) cnt[threadIdx.x] = 0ull;
  __syncthreads();
  const double p0 = probs[4 * i], p1 = probs[4 * i + 1], p2 = probs[4 * i + 2], p3 = probs[4 * i + 3];
  // running sums over the reachable states, in state order
  const double pr[4] = {p0, p1, p2, p3};
  double run[4];
  int last = -1;
  double acc = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (pr[s] > 0.0) {
      acc = acc + pr[s];
      last = s;
    }
    run[s] = acc;
  }
  unsigned long long c[4] = {0ull, 0ull, 0ull, 0ull};
  const int64_t wi = w[i];
  // draws j of prefix i: this block takes j = y * 256 + thread (mod 256 gridDim.y)
  const int64_t stride = (int64_t)blockDim.x * gridDim.y;
  for (int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; j < wi; j += stride) {
    const double u = bas_uniform((uint32_t)j, (uint32_t)i, (uint32_t)k, seed);
    int cat = last;
#pragma unroll
    for (int s = 3; s >= 0; --s)
      if (pr[s] > 0.0 && u < run[s]) cat = s;
    if (cat >= 0) c[cat]++;
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
    if (c[s]) atomicAdd(&cnt[s], c[s]);
  __syncthreads();
  if (threadIdx.x < 4) {
    if (gridDim.y == 1) counts[4 * i + threadIdx.x] = (int64_t)cnt[threadIdx.x];
    else if (cnt[threadIdx.x]) atomicAdd((unsigned long long*)&counts[4 * i + threadIdx.x], cnt[threadIdx.x]);
  }
}

__global__ void k_bas_zero(int64_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Exclusive scan of the prefix weights within blocks of 1024 (woff), and the block totals.
__global__ void __launch_bounds__(1024) k_bas_wscan_blocks(const int64_t* __restrict__ w, int64_t U,
                                                           int64_t* __restrict__ woff, int64_t* __restrict__ btot) {
  __shared__ int64_t s[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int64_t v = i < U ? w[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int64_t t = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < U) woff[i] = s[threadIdx.x] - v;
  if (threadIdx.x == 1023) btot[blockIdx.x] = s[1023];
}

// Draw counts over the flat draw index: draw j of the step belongs to the prefix i whose
// weight range [off_i, off_i + w_i) holds j (off: block offsets boff, then woff within the
// block), and is draw j - off_i of that prefix, so it uses the same uniform as in
// k_bas_counts. Many prefixes with few draws each then cost one thread per draw instead of
// one block per prefix. A wave whose draws all fall in one prefix adds its four counts once;
// otherwise every draw adds 1 (integer atomics: the totals do not depend on their order).
__global__ void __launch_bounds__(256) k_bas_counts_flat(const double* __restrict__ probs,
                                                         const int64_t* __restrict__ woff,
                                                         const int64_t* __restrict__ boff, int64_t nblk, int64_t U,
                                                         const int64_t* __restrict__ total, int k, uint64_t seed,
                                                         int64_t* __restrict__ counts) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = *total;
  const bool live = j < N;
  int64_t i = 0, jl = 0;
  int cat = -1;
  if (live) {
    // block: the last b with boff[b] <= j (boff ascending, boff[0] = 0)
    int64_t lo = 0, hi = nblk - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (boff[mid] <= j) lo = mid; else hi = mid - 1;
    }
    const int64_t b = lo, r = j - boff[b];
    int64_t l0 = b * 1024, l1 = (b * 1024 + 1023 < U ? b * 1024 + 1023 : U - 1);
    while (l0 < l1) {
      const int64_t mid = (l0 + l1 + 1) >> 1;
      if (woff[mid] <= r) l0 = mid; else l1 = mid - 1;
    }
    i = l0;
    jl = r - woff[i];
    const double p0 = probs[4 * i], p1 = probs[4 * i + 1], p2 = probs[4 * i + 2], p3 = probs[4 * i + 3];
    const double pr[4] = {p0, p1, p2, p3};
    double run[4];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (pr[q] > 0.0) {
        acc = acc + pr[q];
        cat = q;
      }
      run[q] = acc;
    }
    const double u = bas_uniform((uint32_t)jl, (uint32_t)i, (uint32_t)k, seed);
#pragma unroll
    for (int q = 3; q >= 0; --q)
      if (pr[q] > 0.0 && u < run[q]) cat = q;
  }
  const int64_t i0 = __shfl(i, 0);
  const uint64_t act = __ballot(live && cat >= 0);
  if (__ballot(live && cat >= 0 && i == i0) == act) {   // one prefix for the whole wave
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t m = __ballot(live && cat == q);
      if (lane == 0 && m) atomicAdd((unsigned long long*)&counts[4 * i0 + q], (unsigned long long)__popcll(m));
    }
  } else if (live && cat >= 0) {
    atomicAdd((unsigned long long*)&counts[4 * i + cat], 1ull);
  }
}

// Number of surviving children per prefix, and their exclusive scan (blocks of 1024,
// then the block totals, then the block offsets added).
__global__ void __launch_bounds__(1024) k_bas_scan_blocks(const int64_t* __restrict__ counts, int64_t U,
                                                          int64_t* __restrict__ off, int64_t* __restrict__ btot) {
  __shared__ int64_t s[1024];
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
                                                          int64_t* __restrict__ total) {
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
  if (threadIdx.x == 0) *total = carry;
}

template <int NW>
__global__ void k_bas_emit(const uint64_t* __restrict__ pre, const int64_t* __restrict__ counts, int64_t U, int k,
                           const int64_t* __restrict__ off, const int64_t* __restrict__ btot,
                           uint64_t* __restrict__ child, int64_t* __restrict__ cw, int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= U) return;
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

// ----------------------------------------------------------------------------- launchers
hipError_t launch_bas_step(const SysDev& S, const MadeDev& M, int hmax, const uint64_t* pre, const int64_t* w,
                           int64_t U, int k, uint64_t seed, double* probs, int64_t* counts, int64_t* off,
                           int64_t* btot, int64_t* total, uint64_t* child, int64_t* cw, int64_t cap, int64_t ndraws,
                           hipStream_t st) {
  if (U <= 0 || ndraws <= 0) return hipErrorInvalidValue;
  hipError_t e = launch_bas_probs(S, M, hmax, pre, U, k, probs, st);
  if (e != hipSuccess) return e;
  // few prefixes (the first orbitals) carry all the draws: their draws are spread over up
  // to 64 blocks each, whose integer counts are added atomically (order-independent)
  const unsigned ysplit = U >= 2048 ? 1u : (unsigned)(2048 / U < 64 ? 2048 / U : 64);
  const int64_t nblk = (U + 1023) / 1024;
  hipLaunchKernelGGL(k_bas_zero, dim3((unsigned)((4 * U + 255) / 256)), dim3(256), 0, st, counts, 4 * U);
  if (U < 2048) {
    hipLaunchKernelGGL(k_bas_counts, dim3((unsigned)U, ysplit), dim3(256), 0, st, probs, w, k, seed, counts);
  } else {
    // many prefixes: one thread per draw over the flat draw index (off, btot and total are
    // free until the children's scan below)
    hipLaunchKernelGGL(k_bas_wscan_blocks, dim3((unsigned)nblk), dim3(1024), 0, st, w, U, off, btot);
    hipLaunchKernelGGL(k_bas_scan_totals, dim3(1), dim3(1024), 0, st, btot, nblk, total);
    hipLaunchKernelGGL(k_bas_counts_flat, dim3((unsigned)((ndraws + 255) / 256)), dim3(256), 0, st, probs, off, btot,
                       nblk, U, total, k, seed, counts);
  }
  hipLaunchKernelGGL(k_bas_scan_blocks, dim3((unsigned)nblk), dim3(1024), 0, st, counts, U, off, btot);
  hipLaunchKernelGGL(k_bas_scan_totals, dim3(1), dim3(1024), 0, st, btot, nblk, total);
  if (S.W == 1)
    hipLaunchKernelGGL(k_bas_emit<1>, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, st, pre, counts, U, k, off, btot,
                       child, cw, cap);
  else
    hipLaunchKernelGGL(k_bas_emit<2>, dim3((unsigned)((U + 255) / 256)), dim3(256), 0, st, pre, counts, U, k, off, btot,
                       child, cw, cap);
  return hipGetLastError();
}

}  // namespace elocal
