// Full-sector vectors and the Chebyshev (KPM) recursion on them.
//
// A vector of the (n_alpha, n_beta) sector has one entry per determinant, at index
// r = rank(alpha set) * C(n, n_beta) + rank(beta set), where a set of occupied spatial
// orbitals o_1 < ... < o_k has the combinatorial-number-system rank sum_i C(o_i, i).
// H v is formed row by row ("pull"): one wave per row unranks the row's determinant,
// builds its occupied/virtual lists and single-excitation values in LDS, walks the
// row's canonical connected list (the same generator and Slater--Condon values as the
// local-energy path), ranks every x' and gathers v there. The row's sum, a fixed xor
// tree over the wave, is bitwise repeatable; nothing per row is stored in HBM.
#include "elocal_internal.hpp"
#include "kernels.hpp"

namespace elocal {

// Determinant of rank (ra, rb): greedy unranking of each spin's set.
template <int NW>
__device__ __forceinline__ void sector_unrank(const uint32_t* __restrict__ binom, int n, int na, int nb,
                                              uint32_t ra, uint32_t rb, uint64_t (&x)[NW]) {
#pragma unroll
  for (int w = 0; w < NW; ++w) x[w] = 0;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    uint32_t r = s ? rb : ra;
    int o = n - 1;
    for (int i = s ? nb : na; i >= 1; --i) {
      while (binom[o * 65 + i] > r) --o;
      r -= binom[o * 65 + i];
      const int k = 2 * o + s;
      x[k >> 6] |= 1ull << (k & 63);
      --o;
    }
  }
}

// Rank of one spin's set of occupied orbitals (ascending set bits).
template <int NW>
__device__ __forceinline__ uint32_t spin_rank(const uint32_t* __restrict__ binom, const uint64_t (&x)[NW], int s) {
  const uint64_t pat = s ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull;
  uint32_t r = 0;
  int i = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    uint64_t m = x[w] & pat;
    while (m) {
      const int k = 64 * w + __ffsll((unsigned long long)m) - 1;
      ++i;
      r += binom[(k >> 1) * 65 + i];
      m &= m - 1;
    }
  }
  return r;
}

// One single excitation of a row: the change of its spin's rank and (I, A, parity of
// the single applied alone).
struct KpmSingle {
  int32_t drank;
  uint32_t info;   // I | A << 8 | parity << 16
};

// y = ch (H v) + cv v + cz z over the whole sector (z may be null); per wave, the
// partial sums of y.y and y.v over its rows (fixed row order) go to partial[wave].
// LDS per wave (stride `wstride` bytes): the row's SampleCtx, its nSa + nSb
// single-excitation values, then its table of single excitations; after the four wave
// areas, rows 0..n-1 of the binomial table. Singles and
// opposite-spin doubles (an alpha single u1 with a beta single u2) come from the table:
// x' has rank (ra + drank(u1)) C(n, n_beta) + rb + drank(u2), and applying a_I, a_J, a+_B,
// a+_A in that order has parity par(u1) + par(u2) + [I < J] + [I < B] + [J < A] + [B < A]
// (each later operator also counts the orbitals the earlier ones emptied or filled below
// it). The same-spin doubles go through the generator and rank only their spin.
template <int NW>
__global__ void __launch_bounds__(256) k_sector_apply(SysDev S, const uint32_t* __restrict__ binom, int64_t dim,
                                                      uint32_t nb_dim, double ch, double cv,
                                                      const double* __restrict__ v, double cz,
                                                      const double* __restrict__ z, double* __restrict__ y,
                                                      double* __restrict__ partial, uint32_t wstride) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t nS = S.nSa + S.nSb;
  struct {
    SampleCtx& c;
    double* F;
    KpmSingle* T;
  } wc{*(SampleCtx*)(smem + wid * wstride), (double*)(smem + wid * wstride + sizeof(SampleCtx)),
       (KpmSingle*)(smem + wid * wstride + sizeof(SampleCtx) + 8u * nS)};
  const uint32_t ab0 = 1u + nS + S.nDaa + S.nDbb;   // first opposite-spin double
  const int n = S.n;
  // rows 0..n-1 of the binomial table in LDS (after the four wave areas): the rankings read
  // it inside data-dependent loops, where every global load would be waited for in turn
  uint32_t* sbin = (uint32_t*)(smem + 4u * wstride);
  for (uint32_t i = threadIdx.x; i < (uint32_t)n * 65u; i += blockDim.x) sbin[i] = binom[i];
  __syncthreads();
  const int64_t wave = (int64_t)blockIdx.x * 4 + wid, nwaves = (int64_t)gridDim.x * 4;
  double yy = 0.0, yv = 0.0;
  for (int64_t r = wave; r < dim; r += nwaves) {
    const uint32_t ra = (uint32_t)(r / nb_dim), rb = (uint32_t)(r % nb_dim);
    uint64_t x[NW];
    sector_unrank<NW>(sbin, S.n, S.na, S.nb, ra, rb, x);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    build_ctx<NW>(S, x, wc.c, lane);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double ed = sample_terms<NW>(S, x, wc.c, lane, wc.F);
    for (uint32_t u = lane; u < nS; u += 64) {
      const int spin = u >= S.nSa;
      const uint32_t w = spin ? u - S.nSa : u;
      const uint32_t q = spin ? fdiv(w, S.f_vb) : fdiv(w, S.f_va);
      const int I = 2 * wc.c.occ[spin][q] + spin, A = 2 * wc.c.vir[spin][w - q * (spin ? S.vb : S.va)] + spin;
      uint64_t y1[NW];
#pragma unroll
      for (int k = 0; k < NW; ++k) y1[k] = x[k];
      int par = parity_below<NW>(y1, I);
      flip<NW>(y1, I);
      par ^= parity_below<NW>(y1, A);
      flip<NW>(y1, A);
      wc.T[u].drank = (int32_t)spin_rank<NW>(sbin, y1, spin) - (int32_t)(spin ? rb : ra);
      wc.T[u].info = (uint32_t)I | ((uint32_t)A << 8) | ((uint32_t)par << 16);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double acc = 0.0;
    for (uint32_t t0 = 0; t0 < S.C; t0 += 64) {
      const uint32_t t = t0 + lane;
      if (t < S.C) {
        double val;
        int neg;
        int64_t idx;
        if (t >= ab0) {
          const uint32_t u = t - ab0, u1 = fdiv(u, S.f_nSb), u2 = S.nSa + (u - u1 * S.nSb);
          const KpmSingle sa = wc.T[u1], sb = wc.T[u2];
          const int I = sa.info & 0xFF, A = (sa.info >> 8) & 0xFF, J = sb.info & 0xFF, Bq = (sb.info >> 8) & 0xFF;
          neg = (int)(((sa.info ^ sb.info) >> 16) & 1u) ^ (I < J) ^ (I < Bq) ^ (J < A) ^ (Bq < A);
          val = S.S[((((size_t)(I >> 1) * n + (J >> 1)) * n + (A >> 1)) * n) + (Bq >> 1)];
          idx = (int64_t)((int64_t)ra + sa.drank) * nb_dim + ((int64_t)rb + sb.drank);
        } else if (t >= 1u && t < 1u + nS) {
          const uint32_t u = t - 1u;
          const KpmSingle sg = wc.T[u];
          neg = (int)((sg.info >> 16) & 1u);
          val = wc.F[u];
          idx = u < S.nSa ? ((int64_t)ra + sg.drank) * nb_dim + rb : (int64_t)ra * nb_dim + ((int64_t)rb + sg.drank);
        } else if (t == 0u) {
          neg = 0;
          val = ed;
          idx = r;
        } else {   // same-spin double: only that spin's set changes
          const Excitation e = unrank(S, wc.c, t);
          uint64_t xo[NW];
          neg = apply_excitation<NW>(x, e, xo) < 0;
          val = excitation_value(S, e, wc.F, ed);
          idx = e.spin == 0 ? (int64_t)spin_rank<NW>(sbin, xo, 0) * nb_dim + rb
                            : (int64_t)ra * nb_dim + spin_rank<NW>(sbin, xo, 1);
        }
        acc += (neg ? -val : val) * v[idx];
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    const double vr = v[r];
    double yr = ch * acc + cv * vr;
    if (z) yr += cz * z[r];
    if (lane == 0) y[r] = yr;
    yy += yr * yr;
    yv += yr * vr;
  }
  if (lane == 0) {
    partial[2 * wave] = yy;
    partial[2 * wave + 1] = yv;
  }
}

// Basis enumeration: x[r] for every r (one thread per row).
template <int NW>
__global__ void k_sector_basis(SysDev S, const uint32_t* __restrict__ binom, int64_t dim, uint32_t nb_dim,
                               uint64_t* __restrict__ x) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= dim) return;
  uint64_t w[NW];
  sector_unrank<NW>(binom, S.n, S.na, S.nb, (uint32_t)(r / nb_dim), (uint32_t)(r % nb_dim), w);
#pragma unroll
  for (int k = 0; k < NW; ++k) x[r * NW + k] = w[k];
}

// Sum of the per-wave partials in a fixed tree (one block); then, for the KPM recursion,
// the moments of step n (Omega_{2n+1} = 2 <a_{n+1}|a_n> - Omega_1, Omega_{2n+2} =
// 2 <a_{n+1}|a_{n+1}> - Omega_0) or, for n < 0, just the two sums into dots.
__global__ void __launch_bounds__(1024) k_sector_dots(const double* __restrict__ partial, int64_t nw,
                                                      double* __restrict__ dots, double* __restrict__ mu,
                                                      int64_t n, int64_t n_moments) {
  __shared__ double s0[1024], s1[1024];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < nw; i += 1024) {
    a += partial[2 * i];
    b += partial[2 * i + 1];
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int off = 512; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double yy = s0[0], yv = s1[0];
    if (dots) {
      dots[0] = yy;
      dots[1] = yv;
    }
    if (mu) {
      if (n == 0) {            // y = a_1 = H~ a_0: Omega_1 = <a_1|a_0>, Omega_2 = 2 <a_1|a_1> - Omega_0
        if (1 < n_moments) mu[1] = yv;
        if (2 < n_moments) mu[2] = 2.0 * yy - mu[0];
      } else {                 // y = a_{n+1}
        if (2 * n + 1 < n_moments) mu[2 * n + 1] = 2.0 * yv - mu[1];
        if (2 * n + 2 < n_moments) mu[2 * n + 2] = 2.0 * yy - mu[0];
      }
    }
  }
}

// Omega_0 = <a_0|a_0> (fixed tree, one block).
__global__ void __launch_bounds__(1024) k_norm2(const double* __restrict__ v, int64_t dim, double* __restrict__ out) {
  __shared__ double s[1024];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < dim; i += 1024) a += v[i] * v[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int off = 512; off >= 1; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

// Jackson-damped line shape: rho(w) = [g_0 Omega_0 + 2 sum_n g_n Omega_n T_n(w)] /
// (pi sqrt(1 - w^2)), T_n by the three-term recurrence; one thread per point.
__global__ void k_line_shape(const double* __restrict__ mu, int64_t N, const double* __restrict__ w, int64_t P,
                             double* __restrict__ rho) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  const double x = w[j];
  const double q = M_PI / (double)(N + 1), cq = cos(q) / sin(q);
  double t_prev = 1.0, t_cur = x;
  double s = mu[0];   // g_0 = 1
  for (int64_t n = 1; n < N; ++n) {
    double sn, cn;
    sincospi((double)n / (double)(N + 1), &sn, &cn);
    const double g = ((double)(N - n + 1) * cn + sn * cq) / (double)(N + 1);
    s += 2.0 * g * mu[n] * t_cur;
    const double t_next = 2.0 * x * t_cur - t_prev;
    t_prev = t_cur;
    t_cur = t_next;
  }
  rho[j] = s / (M_PI * sqrt(1.0 - x * x));
}

// Pauli-string route: the identity-flip group (diagonal strings) of every sample,
// ediag[b] = sum_k c_k (-1)^|z_k & x_b| in string order; one thread per sample.
__global__ void k_pauli_diag(const uint64_t* __restrict__ x, int64_t B, const uint32_t* __restrict__ off,
                             const uint64_t* __restrict__ z, const double* __restrict__ coef,
                             double* __restrict__ ediag) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint64_t xb = x[b];
  double h = 0.0;
  for (uint32_t k = off[0], e = off[1]; k < e; ++k) h += (__popcll(z[k] & xb) & 1) ? -coef[k] : coef[k];
  ediag[b] = h;
}

// ----------------------------------------------------------------------------- launchers
hipError_t launch_pauli_diag(const uint64_t* x, int64_t B, const uint32_t* off, const uint64_t* z,
                             const double* coef, double* ediag, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pauli_diag, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, x, B, off, z, coef, ediag);
  return hipGetLastError();
}

hipError_t launch_sector_apply(const SysDev& S, const uint32_t* binom, int64_t dim, uint32_t nb_dim, double ch,
                               double cv, const double* v, double cz, const double* z, double* y, double* partial,
                               unsigned grid, hipStream_t st) {
  if (dim <= 0) return hipSuccess;
  const uint32_t nS = S.nSa + S.nSb;
  // per wave: SampleCtx, nS single values (8 B), nS table rows (8 B)
  const uint32_t wstride = (uint32_t)((sizeof(SampleCtx) + 16u * (nS ? nS : 1u) + 15u) & ~15u);
  const size_t lds = 4u * wstride + (size_t)S.n * 65u * sizeof(uint32_t);   // + binomial rows
  if (lds > 65536) {
    auto kern = (S.W == 1) ? (const void*)k_sector_apply<1> : (const void*)k_sector_apply<2>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (S.W == 1)
    hipLaunchKernelGGL(k_sector_apply<1>, dim3(grid), dim3(256), lds, st, S, binom, dim, nb_dim, ch, cv, v, cz, z, y,
                       partial, wstride);
  else
    hipLaunchKernelGGL(k_sector_apply<2>, dim3(grid), dim3(256), lds, st, S, binom, dim, nb_dim, ch, cv, v, cz, z, y,
                       partial, wstride);
  return hipGetLastError();
}

hipError_t launch_sector_dots(const double* partial, int64_t nw, double* dots, double* mu, int64_t n,
                              int64_t n_moments, hipStream_t st) {
  hipLaunchKernelGGL(k_sector_dots, dim3(1), dim3(1024), 0, st, partial, nw, dots, mu, n, n_moments);
  return hipGetLastError();
}

hipError_t launch_norm2(const double* v, int64_t dim, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, st, v, dim, out);
  return hipGetLastError();
}

hipError_t launch_sector_basis(const SysDev& S, const uint32_t* binom, int64_t dim, uint32_t nb_dim, uint64_t* x,
                               hipStream_t st) {
  if (dim <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((dim + 255) / 256);
  if (S.W == 1) hipLaunchKernelGGL(k_sector_basis<1>, dim3(blocks), dim3(256), 0, st, S, binom, dim, nb_dim, x);
  else hipLaunchKernelGGL(k_sector_basis<2>, dim3(blocks), dim3(256), 0, st, S, binom, dim, nb_dim, x);
  return hipGetLastError();
}

hipError_t launch_line_shape(const double* mu, int64_t N, const double* w, int64_t P, double* rho, hipStream_t st) {
  if (P <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_line_shape, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, mu, N, w, P, rho);
  return hipGetLastError();
}

}  // namespace elocal
