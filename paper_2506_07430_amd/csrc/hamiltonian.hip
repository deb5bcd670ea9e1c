// Integral tables, per-sample diagonal/single terms, the materialised connected list
// and the sample check.
#include "elocal_internal.hpp"
#include "kernels.hpp"

namespace elocal {

// S[i][j][a][b] = (ai|bj) so that, for one occupied pair (i, j), the virtual pair (a, b)
// runs contiguously; J2, K2, J3, K3 are the Coulomb/exchange slices used by the
// diagonal and single-excitation values.
__global__ void k_build_tables(int n, const double* __restrict__ eri, double* __restrict__ S,
                               double* __restrict__ J2, double* __restrict__ K2,
                               double* __restrict__ J3, double* __restrict__ K3) {
  const size_t n2 = (size_t)n * n, n3 = n2 * n, n4 = n3 * n;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < n4) {
    const size_t b = tid % n, a = (tid / n) % n, j = (tid / n2) % n, i = tid / n3;
    S[tid] = eri[((a * n + i) * n + b) * n + j];
  }
  if (tid < n3) {
    const size_t p = tid % n, i = (tid / n) % n, a = tid / n2;
    J3[tid] = eri[((a * n + i) * n + p) * n + p];
    K3[tid] = eri[((a * n + p) * n + p) * n + i];
  }
  if (tid < n2) {
    const size_t q = tid % n, p = tid / n;
    J2[tid] = eri[((p * n + p) * n + q) * n + q];
    K2[tid] = eri[((p * n + q) * n + q) * n + p];
  }
}

template <int NW>
__device__ __forceinline__ void load_x(const uint64_t* __restrict__ x, int64_t b, uint64_t (&xv)[NW]) {
#pragma unroll
  for (int w = 0; w < NW; ++w) xv[w] = x[b * NW + w];
}

// One wave per sample (per-sample terms: see sample_terms in elocal_internal.hpp).
template <int NW>
__global__ void __launch_bounds__(256) k_prep(SysDev S, const uint64_t* __restrict__ x, int64_t B,
                                              double* __restrict__ ediag, double* __restrict__ F) {
  __shared__ SampleCtx ctxs[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t b = (int64_t)blockIdx.x * 4 + wid;
  if (b >= B) return;
  SampleCtx& c = ctxs[wid];
  uint64_t xv[NW];
  load_x<NW>(x, b, xv);
  build_ctx<NW>(S, xv, c, lane);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  const double e = sample_terms<NW>(S, xv, c, lane, F + (size_t)b * (S.nSa + S.nSb));
  if (lane == 0) ediag[b] = e;
}

// One thread per list entry: unrank, apply the operators, look up the value, store.
// The four output streams are written with nontemporal stores: they are consumed later,
// and allocating them in L2 would evict the integral tables every entry reads.
template <int NW>
__global__ void __launch_bounds__(256) k_connect(SysDev S, const uint64_t* __restrict__ x,
                                                 int64_t B, uint32_t chunks,
                                                 const double* __restrict__ ediag,
                                                 const double* __restrict__ F,
                                                 uint64_t* __restrict__ xp, double* __restrict__ hval,
                                                 int8_t* __restrict__ sign, uint32_t* __restrict__ exc) {
  __shared__ SampleCtx c;
  const int64_t b = blockIdx.x / chunks;
  const uint32_t chunk = blockIdx.x % chunks;
  uint64_t xv[NW];
  load_x<NW>(x, b, xv);
  if (threadIdx.x < 64) build_ctx<NW>(S, xv, c, threadIdx.x);
  __syncthreads();
  const uint32_t t = chunk * 256u + threadIdx.x;
  if (t >= S.C) return;
  const Excitation e = unrank(S, c, t);
  uint64_t y[NW];
  const int sg = apply_excitation<NW>(xv, e, y);
  const uint32_t nS = S.nSa + S.nSb;
  const double v = excitation_value(S, e, F + (size_t)b * nS, ediag[b]);
  const size_t o = (size_t)b * S.C + t;
#pragma unroll
  for (int w = 0; w < NW; ++w) __builtin_nontemporal_store(y[w], xp + o * NW + w);
  __builtin_nontemporal_store(sg < 0 ? -v : v, hval + o);
  __builtin_nontemporal_store((int8_t)sg, sign + o);
  const uint32_t code = (uint32_t)(e.I < 0 ? 0xFF : e.I) | ((uint32_t)(e.J < 0 ? 0xFF : e.J) << 8) |
                        ((uint32_t)(e.A < 0 ? 0xFF : e.A) << 16) | ((uint32_t)(e.Bq < 0 ? 0xFF : e.Bq) << 24);
  __builtin_nontemporal_store(code, exc + o);
}

__global__ void k_zero_u64(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

template <int NW>
__global__ void k_check(SysDev S, const uint64_t* __restrict__ x, int64_t B, unsigned long long* bad) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  uint64_t xv[NW];
  load_x<NW>(x, b, xv);
  int na = 0, nb = 0;
  for (int p = 0; p < S.n; ++p) { na += getbit<NW>(xv, 2 * p); nb += getbit<NW>(xv, 2 * p + 1); }
  int extra = 0;
  const int N = 2 * S.n;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int lo = 64 * w;
    uint64_t keep = (N >= lo + 64) ? ~0ull : ((N <= lo) ? 0ull : ((1ull << (N - lo)) - 1ull));
    extra += __popcll(xv[w] & ~keep);
  }
  if (na != S.na || nb != S.nb || extra) atomicAdd(bad, 1ull);
}

// ----------------------------------------------------------------------------- launchers
hipError_t launch_build_tables(int n, const double* eri, double* S, double* J2, double* K2,
                               double* J3, double* K3, hipStream_t st) {
  const size_t n4 = (size_t)n * n * n * n;
  const unsigned blocks = (unsigned)((n4 + 255) / 256);
  hipLaunchKernelGGL(k_build_tables, dim3(blocks), dim3(256), 0, st, n, eri, S, J2, K2, J3, K3);
  return hipGetLastError();
}

hipError_t launch_prep(const SysDev& S, const uint64_t* x, int64_t B, double* ediag, double* F,
                       hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((B + 3) / 4);
  if (S.W == 1) hipLaunchKernelGGL(k_prep<1>, dim3(blocks), dim3(256), 0, st, S, x, B, ediag, F);
  else hipLaunchKernelGGL(k_prep<2>, dim3(blocks), dim3(256), 0, st, S, x, B, ediag, F);
  return hipGetLastError();
}

hipError_t launch_connect(const SysDev& S, const uint64_t* x, int64_t B, const double* ediag,
                          const double* F, uint64_t* xp, double* hval, int8_t* sign, uint32_t* exc,
                          hipStream_t st) {
  if (B <= 0) return hipSuccess;
  const uint32_t chunks = (S.C + 255u) / 256u;
  const uint64_t blocks = (uint64_t)B * chunks;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  if (S.W == 1)
    hipLaunchKernelGGL(k_connect<1>, dim3((unsigned)blocks), dim3(256), 0, st, S, x, B, chunks, ediag, F, xp, hval, sign, exc);
  else
    hipLaunchKernelGGL(k_connect<2>, dim3((unsigned)blocks), dim3(256), 0, st, S, x, B, chunks, ediag, F, xp, hval, sign, exc);
  return hipGetLastError();
}

hipError_t launch_check(const SysDev& S, const uint64_t* x, int64_t B, unsigned long long* bad,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, bad, 1);
  if (B > 0) {
    const unsigned blocks = (unsigned)((B + 255) / 256);
    if (S.W == 1) hipLaunchKernelGGL(k_check<1>, dim3(blocks), dim3(256), 0, st, S, x, B, bad);
    else hipLaunchKernelGGL(k_check<2>, dim3(blocks), dim3(256), 0, st, S, x, B, bad);
  }
  return hipGetLastError();
}

}  // namespace elocal
