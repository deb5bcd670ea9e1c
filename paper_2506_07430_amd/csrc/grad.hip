// Local-energy assembly from per-item partials, energy statistics, and the VMC
// gradient: forward recomputation at the samples, hand-written backward, FP64.
// Every reduction runs in a fixed order (no floating-point atomics), so results are
// bitwise repeatable.
#include "elocal_internal.hpp"
#include <algorithm>
#include <cstring>

#include "kernels.hpp"

namespace elocal {

__global__ void k_reduce(const double* __restrict__ ediag, const double* __restrict__ partial,
                         int64_t B, uint32_t ips, double* __restrict__ eloc) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double re = ediag[b], im = 0.0;
  const double* p = partial + 2 * (size_t)b * ips;
  for (uint32_t s = 0; s < ips; ++s) {
    re += p[2 * s];
    im += p[2 * s + 1];
  }
  eloc[2 * b] = re;
  eloc[2 * b + 1] = im;
}

// One block of 1024 threads: strided per-thread sums, then a fixed LDS tree.
__global__ void __launch_bounds__(1024) k_stats(const double* __restrict__ eloc,
                                                const double* __restrict__ w, int64_t B,
                                                double* __restrict__ stats) {
  __shared__ double s0[1024], s1[1024], s2[1024];
  const int t = threadIdx.x;
  double sw = 0.0, sr = 0.0, si = 0.0;
  for (int64_t i = t; i < B; i += 1024) {
    sw += w[i];
    sr += w[i] * eloc[2 * i];
    si += w[i] * eloc[2 * i + 1];
  }
  s0[t] = sw; s1[t] = sr; s2[t] = si;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if (t < h) { s0[t] += s0[t + h]; s1[t] += s1[t + h]; s2[t] += s2[t + h]; }
    __syncthreads();
  }
  const double W = s0[0], er = s1[0] / W, ei = s2[0] / W;
  __syncthreads();
  double sv = 0.0;
  for (int64_t i = t; i < B; i += 1024) {
    const double dr = eloc[2 * i] - er, di = eloc[2 * i + 1] - ei;
    sv += w[i] * (dr * dr + di * di);
  }
  s0[t] = sv;
  __syncthreads();
  for (int h = 512; h >= 1; h >>= 1) {
    if (t < h) s0[t] += s0[t + h];
    __syncthreads();
  }
  if (t == 0) {
    stats[0] = er; stats[1] = ei; stats[2] = s0[0] / W; stats[3] = W;
  }
}

// ----------------------------------------------------------------------------- FP64 GEMM
// C[z][m][n] = sum_{k in chunk z} A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn], on the FP64 matrix cores (v_mfma_f64_16x16x4f64): 64x64
// block tiles staged through LDS 16 k at a time, four waves of 32x32 (2x2 MFMA tiles).
// Operands: lane l gives A row l%16 / B column l%16 at k = l/16; the result holds row
// 4i + l/16, column l%16 in register i. Epilogue (only when gridDim.z == 1): + bias[n],
// then ReLU if `relu`, then zero where gate[m][n] (same layout as C) is not positive (the
// ReLU derivative of a forward activation). Each output is one fixed-order chain of
// products: repeatable.
// Masked operands: with `t.flags & 1` the block of column tile blockIdx.x contracts only
// over k in [k_lo, k_hi) of that tile (the other products have a zero factor); with
// `t.flags & 2` a block whose first column is at or past n_end[blockIdx.y] is all zero.
struct GemmTiles {
  int32_t k_lo[8], k_hi[8], n_end[8];
  int32_t flags;
};

__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const double* __restrict__ A,
                                              int64_t sam, int64_t sak, const double* __restrict__ Bm,
                                              int64_t sbk, int64_t sbn, double* __restrict__ C,
                                              int64_t ldc, int64_t zstride, int kchunk,
                                              const double* __restrict__ bias, int relu,
                                              const double* __restrict__ gate, GemmTiles t) {
  __shared__ double As[16][65], Bs[16][65];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64, z = blockIdx.z;
  int k_begin = z * kchunk;
  int k_end = min(K, k_begin + kchunk);
  if (t.flags & 1) {
    k_begin = max(k_begin, t.k_lo[blockIdx.x]);
    k_end = min(k_end, t.k_hi[blockIdx.x]);
  }
  if ((t.flags & 2) && n0 >= t.n_end[blockIdx.y]) k_end = k_begin;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32, r16 = lane & 15, kq = lane >> 4;
  const bool a_kfast = sak == 1 && sam != 1, b_kfast = sbk == 1 && sbn != 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // each operand is read along its unit-stride index so that a wave's loads coalesce; the
  // next 16-deep slice is fetched into registers while the current one is multiplied
  double ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int mm = a_kfast ? idx >> 4 : idx & 63, kk = a_kfast ? idx & 15 : idx >> 6;
      const int gm = m0 + mm, gk = k0 + kk;
      ra[e] = (gm < M && gk < k_end) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : 0.0;
      const int nn = b_kfast ? idx >> 4 : idx & 63, kb = b_kfast ? idx & 15 : idx >> 6;
      const int gn = n0 + nn, gkb = k0 + kb;
      rb[e] = (gn < N && gkb < k_end) ? Bm[(int64_t)gkb * sbk + (int64_t)gn * sbn] : 0.0;
    }
  };
  if (k_begin < k_end) fetch(k_begin);
  for (int k0 = k_begin; k0 < k_end; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x + 256 * e;
      As[a_kfast ? idx & 15 : idx >> 6][a_kfast ? idx >> 4 : idx & 63] = ra[e];
      Bs[b_kfast ? idx & 15 : idx >> 6][b_kfast ? idx >> 4 : idx & 63] = rb[e];
    }
    __syncthreads();
    if (k0 + 16 < k_end) fetch(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk + kq][wm + 16 * i + r16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + kq][wn + 16 * j + r16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + wm + 16 * i + 4 * q + kq, gn = n0 + wn + 16 * j + r16;
        if (gm >= M || gn >= N) continue;
        double v = acc[i][j][q];
        if (bias) v += bias[gn];
        if (relu && v < 0.0) v = 0.0;
        if (gate && !(gate[(int64_t)gm * ldc + gn] > 0.0)) v = 0.0;
        C[(int64_t)z * zstride + (int64_t)gm * ldc + gn] = v;
      }
}

// out[i] = sum_z part[z][i] in a fixed order: four running sums over z = j mod 4,
// combined pairwise (independent loads in flight instead of one dependent chain).
__global__ void k_sum_splits(const double* __restrict__ part, int splits, int64_t count,
                             double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int z = 0;
  for (; z + 3 < splits; z += 4) {
    s0 += part[(int64_t)z * count + i];
    s1 += part[(int64_t)(z + 1) * count + i];
    s2 += part[(int64_t)(z + 2) * count + i];
    s3 += part[(int64_t)(z + 3) * count + i];
  }
  for (; z < splits; ++z) s0 += part[(int64_t)z * count + i];
  out[i] = (s0 + s1) + (s2 + s3);
}

__device__ __forceinline__ bool grad_allowed(int n, int L, int l, int o, int k) {
  const int nm1 = n - 1;
  if (l == 0) return (o % nm1) + 1 >= k / 2 + 1;
  if (l < L) return (o % nm1) + 1 >= (k % nm1) + 1;
  if (o == 4 * n) return true;
  return (o / 4) + 1 > (k % nm1) + 1;
}

__device__ __forceinline__ double theta_at(int precision, const void* theta, uint32_t i) {
  if (precision == 0) return ((const double*)theta)[i];
  const uint16_t b = ((const uint16_t*)theta)[i];
  return (double)__uint_as_float((uint32_t)b << 16);
}

// Hidden units are held in degree-sorted order in the workspace (position p is the
// caller's unit sorted_unit(n, w, p)), so that every unit's unmasked inputs are a prefix
// of the previous layer: input bits (orbital order) and logits (orbital order, phase row
// last) keep their order.
__device__ __forceinline__ int caller_out(const GradPlan& G, int l, int o) {
  return l < G.L ? sorted_unit(G.n, G.dims[l + 1], o) : o;
}
__device__ __forceinline__ int caller_in(const GradPlan& G, int l, int k) {
  return l > 0 ? sorted_unit(G.n, G.dims[l], k) : k;
}

// Masked FP64 weights [out][in] and biases of every layer; the output layer gets the
// phase head appended as row 4n.
__global__ void k_unpack_masked(GradPlan G) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t base = 0;
  for (int l = 0; l <= G.L; ++l) {
    const int in = G.dims[l], out = G.dims[l + 1];
    const int64_t cnt = (int64_t)out * in + out;
    if (gid < base + cnt) {
      const int64_t r = gid - base;
      if (r < (int64_t)out * in) {
        const int o = caller_out(G, l, (int)(r / in)), k = caller_in(G, l, (int)(r % in));
        double v = 0.0;
        if (grad_allowed(G.n, G.L, l, o, k)) {
          const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offwphi + k : G.T.offW[l] + (uint32_t)o * in + k;
          v = theta_at(G.precision, G.theta, ti);
        }
        G.Wm[l][r] = v;
      } else {
        const int p = (int)(r - (int64_t)out * in), o = caller_out(G, l, p);
        const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offbphi : G.T.offb[l] + o;
        G.bm[l][p] = theta_at(G.precision, G.theta, ti);
      }
      return;
    }
    base += cnt;
  }
}

template <int NW>
__global__ void k_bits(const uint64_t* __restrict__ x, int64_t B, int N, double* __restrict__ h0) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= B * N) return;
  const int64_t b = gid / N;
  const int k = (int)(gid % N);
  h0[gid] = (double)((x[b * NW + (k >> 6)] >> (k & 63)) & 1ull);
}

// Cotangents of the logits and the phase logit, one thread per (sample, orbital) and one
// per sample for the phase:
//   gA = 2 wbar Re(E - <E>), gphi = 2 wbar Im(E - <E>);
//   dz[p][s] = gA/2 ([s == s_p] - softmax_p(s)) on allowed s; dz_phi = gphi 2 pi sig (1 - sig).
// The allowed states of orbital p follow from the electrons placed below it (popcounts).
template <int NW>
__global__ void k_softmax_bwd(const uint64_t* __restrict__ x, const double* __restrict__ w,
                              const double* __restrict__ eloc, const double* __restrict__ stats,
                              int64_t B, int n, int na, int nb, const double* __restrict__ logits,
                              double* __restrict__ dlog) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = gid / (n + 1);
  const int p = (int)(gid - b * (n + 1));
  if (b >= B) return;
  const int O = 4 * n + 1;
  const double wbar = w[b] / stats[3];
  const double* z = logits + b * O;
  double* d = dlog + b * O;
  if (p == n) {
    const double gphi = 2.0 * wbar * (eloc[2 * b + 1] - stats[1]);
    const double sig = 1.0 / (1.0 + exp(-z[4 * n]));
    d[4 * n] = gphi * 2.0 * M_PI * sig * (1.0 - sig);
    return;
  }
  const double gA = 2.0 * wbar * (eloc[2 * b] - stats[0]);
  int cu = 0, cd = 0, s = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const uint64_t v = x[b * NW + q];
    const int below = 2 * p - 64 * q;   // bits of this word that lie below orbital p
    const uint64_t m = below <= 0 ? 0ull : below >= 64 ? ~0ull : ((1ull << below) - 1ull);
    cu += __popcll(v & m & 0x5555555555555555ull);
    cd += __popcll(v & m & 0xAAAAAAAAAAAAAAAAull);
    if (below >= 0 && below < 64) s = (int)((v >> below) & 3ull);
  }
  const int left = n - p - 1;
  bool ok[4];
  double mx = -INFINITY;
  for (int q = 0; q < 4; ++q) {
    const int u = cu + (q & 1), dd = cd + (q >> 1);
    ok[q] = (u <= na) && (dd <= nb) && (u + left >= na) && (dd + left >= nb);
    if (ok[q]) mx = fmax(mx, z[4 * p + q]);
  }
  double e[4], sum = 0.0;
  for (int q = 0; q < 4; ++q) { e[q] = ok[q] ? exp(z[4 * p + q] - mx) : 0.0; sum += e[q]; }
  for (int q = 0; q < 4; ++q)
    d[4 * p + q] = ok[q] ? 0.5 * gA * ((q == s ? 1.0 : 0.0) - e[q] / sum) : 0.0;
}

// part[z][o] = sum of d[b][o] over the rows b of chunk z, in a fixed order (64 columns
// per block; four interleaved row lanes, each with four interleaved running sums, combined
// pairwise at the end).
__global__ void __launch_bounds__(256) k_colsum(const double* __restrict__ d, int64_t B, int out,
                                                int64_t rows, double* __restrict__ part) {
  __shared__ double acc[4][64];
  const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + c;
  const int64_t b0 = (int64_t)blockIdx.y * rows, b1 = min(B, b0 + rows);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (o < out) {
    int64_t b = b0 + r;
    for (; b + 12 < b1; b += 16) {
      s0 += d[b * out + o];
      s1 += d[(b + 4) * out + o];
      s2 += d[(b + 8) * out + o];
      s3 += d[(b + 12) * out + o];
    }
    for (; b < b1; b += 4) s0 += d[b * out + o];
  }
  acc[r][c] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (r == 0 && o < out) part[(int64_t)blockIdx.y * out + o] = (acc[0][c] + acc[1][c]) + (acc[2][c] + acc[3][c]);
}

// Scatter masked dW / db into the caller's flat layout.
__global__ void k_write_dtheta(GradPlan G) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t base = 0;
  for (int l = 0; l <= G.L; ++l) {
    const int in = G.dims[l], out = G.dims[l + 1];
    const int64_t cnt = (int64_t)out * in + out;
    if (gid < base + cnt) {
      const int64_t r = gid - base;
      if (r < (int64_t)out * in) {
        const int o = caller_out(G, l, (int)(r / in)), k = caller_in(G, l, (int)(r % in));
        const double v = grad_allowed(G.n, G.L, l, o, k) ? G.dW[l][r] : 0.0;
        const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offwphi + k : G.T.offW[l] + (uint32_t)o * in + k;
        G.dtheta[ti] = v;
      } else {
        const int p = (int)(r - (int64_t)out * in), o = caller_out(G, l, p);
        const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offbphi : G.T.offb[l] + o;
        G.dtheta[ti] = G.db[l][p];
      }
      return;
    }
    base += cnt;
  }
}

// Copies a small host-side record (passed by value) to device memory, so a call can
// hand per-system descriptors to a kernel without a host buffer or a synchronisation.
struct Words256 {
  uint32_t w[256];
};

__global__ void k_store_words(Words256 src, uint32_t count, uint32_t* __restrict__ dst) {
  for (uint32_t i = threadIdx.x; i < count; i += blockDim.x) dst[i] = src.w[i];
}

// ----------------------------------------------------------------------------- launchers
hipError_t launch_store_bytes(const void* src, size_t bytes, void* dst, hipStream_t st) {
  if (bytes % 4) return hipErrorInvalidValue;
  const uint32_t* s = (const uint32_t*)src;
  uint32_t* d = (uint32_t*)dst;
  size_t words = bytes / 4;
  while (words > 0) {
    const uint32_t cnt = (uint32_t)(words < 256 ? words : 256);
    Words256 w;
    std::memcpy(w.w, s, cnt * 4);
    hipLaunchKernelGGL(k_store_words, dim3(1), dim3(256), 0, st, w, cnt, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    s += cnt;
    d += cnt;
    words -= cnt;
  }
  return hipSuccess;
}

hipError_t launch_reduce(const double* ediag, const double* partial, int64_t B, uint32_t ips,
                         double* eloc, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, ediag, partial, B, ips, eloc);
  return hipGetLastError();
}

hipError_t launch_stats(const double* eloc, const double* w, int64_t B, double* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(1024), 0, st, eloc, w, B, stats);
  return hipGetLastError();
}

static void gemm(int M, int N, int K, const double* A, int64_t sam, int64_t sak, const double* Bm,
                 int64_t sbk, int64_t sbn, double* C, int64_t ldc, const double* bias, int relu,
                 const double* gate, int splits, double* part, const GemmTiles& t, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
  if (splits <= 1 || bias || relu || gate) {
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, M, N, K, A, sam, sak, Bm, sbk, sbn, C, ldc,
                       (int64_t)0, K > 0 ? K : 1, bias, relu, gate, t);
    return;
  }
  const int kchunk = ((K + splits - 1) / splits + 15) / 16 * 16;
  const int nz = (K + kchunk - 1) / kchunk;
  grid.z = nz;
  const int64_t count = (int64_t)M * N;
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, M, N, K, A, sam, sak, Bm, sbk, sbn, part,
                     (int64_t)N, count, kchunk, (const double*)nullptr, 0, (const double*)nullptr, t);
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, part, nz, count, C);
}

// Unmasked inputs of output position o of layer l (a prefix of the layer's inputs in the
// workspace order): bits of orbitals below the unit's degree for layer 0, hidden units of
// degree <= the unit's degree for hidden layers, units of degree <= the orbital index for
// the logits of an orbital, everything for the phase row.
static int kend_of(const GradPlan& G, int l, int o) {
  const int n = G.n, q = n - 1, in = G.dims[l];
  auto count_le = [&](int D) {
    int c = 0;
    for (int r = 0; r < std::min(D, q); ++r) c += (in > r) ? (in - r - 1) / q + 1 : 0;
    return c;
  };
  if (l == G.L) return o == 4 * n ? in : count_le(o / 4);
  const int D = sorted_unit(n, G.dims[l + 1], o) % q + 1;
  return l == 0 ? std::min(in, 2 * D) : count_le(D);
}

hipError_t launch_grad(const GradPlan& G, hipStream_t st) {
  const int L = G.L;
  const int64_t B = G.B;
  int64_t nw = 0;
  for (int l = 0; l <= L; ++l) nw += (int64_t)G.dims[l + 1] * G.dims[l] + G.dims[l + 1];
  hipLaunchKernelGGL(k_unpack_masked, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, G);
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(1024), 0, st, G.eloc, G.w, B, G.stats);
  const int N0 = G.dims[0];
  const int W = (N0 + 63) / 64;
  if (W == 1) hipLaunchKernelGGL(k_bits<1>, dim3((unsigned)((B * N0 + 255) / 256)), dim3(256), 0, st, G.x, B, N0, G.h[0]);
  else hipLaunchKernelGGL(k_bits<2>, dim3((unsigned)((B * N0 + 255) / 256)), dim3(256), 0, st, G.x, B, N0, G.h[0]);
  // Per-layer tiles of the masked products (64-wide tiles; at most 5 along any layer
  // dimension, since widths are <= 256 and the output layer has 4n + 1 <= 257 rows):
  // fwd: column tile of outputs -> inputs [0, max kend); bwd: column tile of inputs ->
  // outputs [first o with kend(o) > tile start, out); dw: row tile of outputs -> inputs
  // below max kend.
  GemmTiles fwd[kMaxLayers], bwd[kMaxLayers], dw[kMaxLayers];
  for (int l = 0; l <= L; ++l) {
    const int in = G.dims[l], out = G.dims[l + 1];
    fwd[l] = GemmTiles{}; bwd[l] = GemmTiles{}; dw[l] = GemmTiles{};
    if ((out + 63) / 64 > 8 || (in + 63) / 64 > 8) continue;
    int ke[4 * kMaxOrb + 1];
    for (int o = 0; o < out; ++o) ke[o] = kend_of(G, l, o);
    for (int tile = 0; tile * 64 < out; ++tile) {
      int mx = 0;
      for (int o = tile * 64; o < std::min(out, tile * 64 + 64); ++o) mx = std::max(mx, ke[o]);
      fwd[l].k_lo[tile] = 0; fwd[l].k_hi[tile] = mx;
      dw[l].n_end[tile] = mx;
    }
    for (int tile = 0; tile * 64 < in; ++tile) {
      int lo = out;
      for (int o = 0; o < out; ++o)
        if (ke[o] > tile * 64) { lo = std::min(lo, o); }
      bwd[l].k_lo[tile] = lo; bwd[l].k_hi[tile] = out;
    }
    fwd[l].flags = 1; bwd[l].flags = 1; dw[l].flags = 2;
  }
  // forward: h[l+1] = act(h[l] Wm[l]^T + b[l]); the last is the logits (+ phase logit)
  for (int l = 0; l <= L; ++l) {
    const int in = G.dims[l], out = G.dims[l + 1];
    gemm((int)B, out, in, G.h[l], in, 1, G.Wm[l], 1, in, G.h[l + 1], out, G.bm[l], l < L ? 1 : 0,
         nullptr, 1, nullptr, fwd[l], st);
  }
  // cotangents of the output layer
  const unsigned sm_blocks = (unsigned)((B * (G.n + 1) + 255) / 256);
  if (W == 1)
    hipLaunchKernelGGL(k_softmax_bwd<1>, dim3(sm_blocks), dim3(256), 0, st, G.x, G.w, G.eloc, G.stats, B, G.n, G.na, G.nb, G.h[L + 1], G.d0);
  else
    hipLaunchKernelGGL(k_softmax_bwd<2>, dim3(sm_blocks), dim3(256), 0, st, G.x, G.w, G.eloc, G.stats, B, G.n, G.na, G.nb, G.h[L + 1], G.d0);
  // backward: d0 holds dz of layer l's output ([B][out]); weights get dz^T h[l]
  double* dcur = G.d0;
  double* dnext = G.d1;
  for (int l = L; l >= 0; --l) {
    const int in = G.dims[l], out = G.dims[l + 1];
    // dW[l][o][k] = sum_b dz[b][o] h[l][b][k]
    gemm(out, in, (int)B, dcur, 1, out, G.h[l], in, 1, G.dW[l], in, nullptr, 0, nullptr, G.splits, G.part,
         dw[l], st);
    // db[l][o] = sum_b dz[b][o]
    {
      // chunks of at least 64 rows, as many as the split buffer holds (at most 64)
      const int64_t cap = std::min<int64_t>(64, (int64_t)G.splits * G.part_per_split / out);
      const int64_t rows = std::max<int64_t>(64, (B + cap - 1) / cap);
      const unsigned nz = (unsigned)std::max<int64_t>(1, (B + rows - 1) / rows);
      hipLaunchKernelGGL(k_colsum, dim3((unsigned)((out + 63) / 64), nz), dim3(256), 0, st, dcur, B, out, rows,
                         nz == 1 ? G.db[l] : G.part);
      if (nz > 1)
        hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((out + 255) / 256)), dim3(256), 0, st, G.part, (int)nz,
                           (int64_t)out, G.db[l]);
    }
    if (l > 0) {
      // dh[b][k] = sum_o dz[b][o] Wm[l][o][k], times ReLU' of layer l-1's output
      gemm((int)B, in, out, dcur, out, 1, G.Wm[l], in, 1, dnext, in, nullptr, 0, G.h[l], 1, nullptr, bwd[l], st);
      double* t = dcur; dcur = dnext; dnext = t;
    }
  }
  hipLaunchKernelGGL(k_write_dtheta, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, G);
  return hipGetLastError();
}

}  // namespace elocal
