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

// One list entry: x' = the excitation applied to x, H_{x x'} with its sign, the sign, and the
// four spin-orbitals of the excitation (0xFF for unused slots), one byte each.
template <int NW>
struct ListEntry {
  uint64_t y[NW];
  double h;
  int8_t sg;
  uint32_t code;
};

template <int NW>
__device__ __forceinline__ ListEntry<NW> list_entry(const SysDev& S, const SampleCtx& c, const uint64_t (&xv)[NW],
                                                    const double* Fs, double ed, uint32_t t) {
  ListEntry<NW> r;
  const Excitation e = unrank(S, c, t);
  const int sg = apply_excitation<NW>(xv, e, r.y);
  const double v = excitation_value(S, e, Fs, ed);
  r.h = sg < 0 ? -v : v;
  r.sg = (int8_t)sg;
  // unused slots hold -1, whose low byte is the 0xFF marker
  r.code = ((uint32_t)e.I & 0xFFu) | (((uint32_t)e.J & 0xFFu) << 8) | (((uint32_t)e.A & 0xFFu) << 16) |
           ((uint32_t)e.Bq << 24);
  return r;
}

// The four output streams are written with nontemporal stores: they are consumed later,
// and allocating them in L2 would evict the integral tables every entry reads.
template <int NW>
__device__ __forceinline__ void store_entry(const ListEntry<NW>& r, size_t o, uint64_t* __restrict__ xp,
                                            double* __restrict__ hval, int8_t* __restrict__ sign,
                                            uint32_t* __restrict__ exc) {
#pragma unroll
  for (int w = 0; w < NW; ++w) __builtin_nontemporal_store(r.y[w], xp + o * NW + w);
  __builtin_nontemporal_store(r.h, hval + o);
  __builtin_nontemporal_store(r.sg, sign + o);
  __builtin_nontemporal_store(r.code, exc + o);
}

// One thread per list entry, scalar stores (outputs of any alignment).
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
  const ListEntry<NW> r = list_entry<NW>(S, c, xv, F + (size_t)b * (S.nSa + S.nSb), ediag[b], t);
  store_entry<NW>(r, (size_t)b * S.C + t, xp, hval, sign, exc);
}

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Two consecutive entries per thread, stored as one vector per stream (16 B of x' per word
// and of H, 8 B of codes, 2 B of signs), over the flat entry index o = b C + t: block k
// takes entries [512 k, 512 k + 512), so every wave writes whole, aligned pieces of each
// stream, which the memory system takes at a much higher rate than one entry per thread
// over per-sample blocks (whose pieces start at arbitrary offsets b C). With C >= 512 a
// block spans at most two samples; waves 0 and 1 build their contexts. A pair starts at an
// even o, so with outputs aligned to 16 (x', H), 8 (codes) and 2 (signs) bytes every vector
// store is naturally aligned.
template <int NW>
__device__ __forceinline__ ListEntry<NW> flat_entry(const SysDev& S, const SampleCtx (&c)[2], int64_t b0,
                                                    const uint64_t* __restrict__ x, const double* __restrict__ ediag,
                                                    const double* __restrict__ F, size_t o) {
  const int64_t b = b0 + (o >= (size_t)(b0 + 1) * S.C ? 1 : 0);
  const uint32_t t = (uint32_t)(o - (size_t)b * S.C);
  uint64_t xv[NW];
  load_x<NW>(x, b, xv);
  return list_entry<NW>(S, c[b - b0], xv, F + (size_t)b * (S.nSa + S.nSb), ediag[b], t);
}

template <int NW>
__global__ void __launch_bounds__(256) k_connect_flat(SysDev S, const uint64_t* __restrict__ x, int64_t B,
                                                      const double* __restrict__ ediag,
                                                      const double* __restrict__ F,
                                                      uint64_t* __restrict__ xp, double* __restrict__ hval,
                                                      int8_t* __restrict__ sign, uint32_t* __restrict__ exc) {
  __shared__ SampleCtx c[2];
  const size_t E = (size_t)B * S.C;
  const size_t o0 = (size_t)blockIdx.x * 512u;
  const int64_t b0 = (int64_t)(o0 / S.C);
  const int wid = threadIdx.x >> 6;
  if (wid < 2 && b0 + wid < B) {
    uint64_t xv[NW];
    load_x<NW>(x, b0 + wid, xv);
    build_ctx<NW>(S, xv, c[wid], threadIdx.x & 63);
  }
  __syncthreads();
  const size_t o = o0 + 2u * threadIdx.x;   // even
  if (o >= E) return;
  if (o + 1u >= E) {
    store_entry<NW>(flat_entry<NW>(S, c, b0, x, ediag, F, o), o, xp, hval, sign, exc);
    return;
  }
  // the pair's sample words, single-excitation row and diagonal are read once; the second
  // entry starts the next sample only when the first is a sample's last
  const int64_t b = b0 + (o >= (size_t)(b0 + 1) * S.C ? 1 : 0);
  const uint32_t t = (uint32_t)(o - (size_t)b * S.C);
  uint64_t xv[NW];
  load_x<NW>(x, b, xv);
  const double* Fs = F + (size_t)b * (S.nSa + S.nSb);
  const double ed = ediag[b];
  const ListEntry<NW> r0 = list_entry<NW>(S, c[b - b0], xv, Fs, ed, t);
  const ListEntry<NW> r1 = t + 1u < S.C ? list_entry<NW>(S, c[b - b0], xv, Fs, ed, t + 1u)
                                        : flat_entry<NW>(S, c, b0, x, ediag, F, o + 1u);
  static_assert(NW == 1 || NW == 2, "one or two words per determinant");
  if constexpr (NW == 1) {
    const u64x2 y = {r0.y[0], r1.y[0]};
    __builtin_nontemporal_store(y, (u64x2*)(xp + o));
  } else {
    const u64x2 y0 = {r0.y[0], r0.y[1]}, y1 = {r1.y[0], r1.y[1]};
    __builtin_nontemporal_store(y0, (u64x2*)(xp + o * NW));
    __builtin_nontemporal_store(y1, (u64x2*)(xp + o * NW + NW));
  }
  const f64x2 h = {r0.h, r1.h};
  __builtin_nontemporal_store(h, (f64x2*)(hval + o));
  const uint16_t sg2 = (uint16_t)((uint8_t)r0.sg | ((uint16_t)(uint8_t)r1.sg << 8));   // byte o = entry o
  __builtin_nontemporal_store(sg2, (uint16_t*)(sign + o));
  const u32x2 cd = {r0.code, r1.code};
  __builtin_nontemporal_store(cd, (u32x2*)(exc + o));
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
  // the flat paired kernel needs outputs aligned to 16 (x', H), 8 (codes) and 2 (signs)
  // bytes, and lists of at least 512 entries (a block then spans at most two samples)
  const bool flat = S.C >= 512u && ((uintptr_t)xp % 16u == 0) && ((uintptr_t)hval % 16u == 0) &&
                    ((uintptr_t)exc % 8u == 0) && ((uintptr_t)sign % 2u == 0);
  if (flat) {
    const uint64_t blocks = ((uint64_t)B * S.C + 511u) / 512u;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (S.W == 1)
      hipLaunchKernelGGL(k_connect_flat<1>, dim3((unsigned)blocks), dim3(256), 0, st, S, x, B, ediag, F, xp, hval, sign, exc);
    else
      hipLaunchKernelGGL(k_connect_flat<2>, dim3((unsigned)blocks), dim3(256), 0, st, S, x, B, ediag, F, xp, hval, sign, exc);
  } else {
    const uint32_t chunks = (S.C + 255u) / 256u;
    const uint64_t blocks = (uint64_t)B * chunks;
    if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (S.W == 1)
      hipLaunchKernelGGL(k_connect<1>, dim3((unsigned)blocks), dim3(256), 0, st, S, x, B, chunks, ediag, F, xp, hval, sign, exc);
    else
      hipLaunchKernelGGL(k_connect<2>, dim3((unsigned)blocks), dim3(256), 0, st, S, x, B, chunks, ediag, F, xp, hval, sign, exc);
  }
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
