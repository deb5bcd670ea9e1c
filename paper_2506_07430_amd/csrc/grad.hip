// Local-energy assembly from per-item partials, energy statistics, and the VMC
// gradient: forward recomputation at the samples, hand-written backward, FP64.
// Every reduction runs in a fixed order (no floating-point atomics), so results are
// bitwise repeatable.
#include "elocal_internal.hpp"
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
// B(k,n) = B[k*sbk + n*sbn]; 64x64 tiles, 16-deep k steps, 4x4 per thread.
// Epilogue (only when gridDim.z == 1): + bias[n], then ReLU if `relu`.
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const double* __restrict__ A,
                                              int64_t sam, int64_t sak, const double* __restrict__ Bm,
                                              int64_t sbk, int64_t sbn, double* __restrict__ C,
                                              int64_t ldc, int64_t zstride, int kchunk,
                                              const double* __restrict__ bias, int relu) {
  __shared__ double As[16][65], Bs[16][65];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64, z = blockIdx.z;
  const int k_begin = z * kchunk;
  const int k_end = min(K, k_begin + kchunk);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = k_begin; k0 < k_end; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = threadIdx.x + 256 * e;
      const int mm = idx & 63, kk = idx >> 6;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < k_end) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : 0.0;
      const int gn = n0 + mm;
      Bs[kk][mm] = (gn < N && gk < k_end) ? Bm[(int64_t)gk * sbk + (int64_t)gn * sbn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) { a[i] = As[kk][ty + 16 * i]; b[i] = Bs[kk][tx + 16 * i]; }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx + 16 * j;
      if (gn >= N) continue;
      double v = acc[i][j];
      if (bias) v += bias[gn];
      if (relu && v < 0.0) v = 0.0;
      C[(int64_t)z * zstride + (int64_t)gm * ldc + gn] = v;
    }
  }
}

// out[i] = sum_z part[z][i] (fixed order).
__global__ void k_sum_splits(const double* __restrict__ part, int splits, int64_t count,
                             double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * count + i];
  out[i] = s;
}

__global__ void k_fill(double* p, int64_t count, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
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
        const int o = (int)(r / in), k = (int)(r % in);
        double v = 0.0;
        if (grad_allowed(G.n, G.L, l, o, k)) {
          const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offwphi + k : G.T.offW[l] + (uint32_t)o * in + k;
          v = theta_at(G.precision, G.theta, ti);
        }
        G.Wm[l][r] = v;
      } else {
        const int o = (int)(r - (int64_t)out * in);
        const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offbphi : G.T.offb[l] + o;
        G.bm[l][o] = theta_at(G.precision, G.theta, ti);
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

// Cotangents of the logits and the phase logit, one thread per sample:
//   gA = 2 wbar Re(E - <E>), gphi = 2 wbar Im(E - <E>);
//   dz[p][s] = gA/2 ([s == s_p] - softmax_p(s)) on allowed s; dz_phi = gphi 2 pi sig (1 - sig).
template <int NW>
__global__ void k_softmax_bwd(const uint64_t* __restrict__ x, const double* __restrict__ w,
                              const double* __restrict__ eloc, const double* __restrict__ stats,
                              int64_t B, int n, int na, int nb, const double* __restrict__ logits,
                              double* __restrict__ dlog) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int O = 4 * n + 1;
  const double wbar = w[b] / stats[3];
  const double gA = 2.0 * wbar * (eloc[2 * b] - stats[0]);
  const double gphi = 2.0 * wbar * (eloc[2 * b + 1] - stats[1]);
  uint64_t xv[NW];
#pragma unroll
  for (int q = 0; q < NW; ++q) xv[q] = x[b * NW + q];
  const double* z = logits + b * O;
  double* d = dlog + b * O;
  int cu = 0, cd = 0;
  for (int p = 0; p < n; ++p) {
    const int left = n - p - 1;
    const int su = getbit<NW>(xv, 2 * p), sd = getbit<NW>(xv, 2 * p + 1);
    const int s = su + 2 * sd;
    bool ok[4];
    double m = -INFINITY;
    for (int q = 0; q < 4; ++q) {
      const int u = cu + (q & 1), dd = cd + (q >> 1);
      ok[q] = (u <= na) && (dd <= nb) && (u + left >= na) && (dd + left >= nb);
      if (ok[q]) m = fmax(m, z[4 * p + q]);
    }
    double e[4], sum = 0.0;
    for (int q = 0; q < 4; ++q) { e[q] = ok[q] ? exp(z[4 * p + q] - m) : 0.0; sum += e[q]; }
    for (int q = 0; q < 4; ++q)
      d[4 * p + q] = ok[q] ? 0.5 * gA * ((q == s ? 1.0 : 0.0) - e[q] / sum) : 0.0;
    cu += su;
    cd += sd;
  }
  const double sig = 1.0 / (1.0 + exp(-z[4 * n]));
  d[4 * n] = gphi * 2.0 * M_PI * sig * (1.0 - sig);
}

// dz = dh where the forward activation was positive (ReLU'), in place.
__global__ void k_relu_bwd(double* __restrict__ d, const double* __restrict__ h, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count && !(h[i] > 0.0)) d[i] = 0.0;
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
        const int o = (int)(r / in), k = (int)(r % in);
        const double v = grad_allowed(G.n, G.L, l, o, k) ? G.dW[l][r] : 0.0;
        const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offwphi + k : G.T.offW[l] + (uint32_t)o * in + k;
        G.dtheta[ti] = v;
      } else {
        const int o = (int)(r - (int64_t)out * in);
        const uint32_t ti = (l == G.L && o == 4 * G.n) ? G.T.offbphi : G.T.offb[l] + o;
        G.dtheta[ti] = G.db[l][o];
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
                 int splits, double* part, hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + 63) / 64, (M + 63) / 64, 1);
  if (splits <= 1 || bias || relu) {
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, M, N, K, A, sam, sak, Bm, sbk, sbn, C, ldc,
                       (int64_t)0, K > 0 ? K : 1, bias, relu);
    return;
  }
  const int kchunk = ((K + splits - 1) / splits + 15) / 16 * 16;
  const int nz = (K + kchunk - 1) / kchunk;
  grid.z = nz;
  const int64_t count = (int64_t)M * N;
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, M, N, K, A, sam, sak, Bm, sbk, sbn, part,
                     (int64_t)N, count, kchunk, (const double*)nullptr, 0);
  hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, part, nz, count, C);
}

hipError_t launch_grad(const GradPlan& G, hipStream_t st) {
  const int L = G.L;
  const int64_t B = G.B;
  int64_t nw = 0;
  for (int l = 0; l <= L; ++l) nw += (int64_t)G.dims[l + 1] * G.dims[l] + G.dims[l + 1];
  hipLaunchKernelGGL(k_unpack_masked, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, G);
  hipLaunchKernelGGL(k_stats, dim3(1), dim3(1024), 0, st, G.eloc, G.w, B, G.stats);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, G.ones, B, 1.0);
  const int N0 = G.dims[0];
  const int W = (N0 + 63) / 64;
  if (W == 1) hipLaunchKernelGGL(k_bits<1>, dim3((unsigned)((B * N0 + 255) / 256)), dim3(256), 0, st, G.x, B, N0, G.h[0]);
  else hipLaunchKernelGGL(k_bits<2>, dim3((unsigned)((B * N0 + 255) / 256)), dim3(256), 0, st, G.x, B, N0, G.h[0]);
  // forward: h[l+1] = act(h[l] Wm[l]^T + b[l]); the last is the logits (+ phase logit)
  for (int l = 0; l <= L; ++l) {
    const int in = G.dims[l], out = G.dims[l + 1];
    gemm((int)B, out, in, G.h[l], in, 1, G.Wm[l], 1, in, G.h[l + 1], out, G.bm[l], l < L ? 1 : 0, 1,
         nullptr, st);
  }
  // cotangents of the output layer
  if (W == 1)
    hipLaunchKernelGGL(k_softmax_bwd<1>, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, G.x, G.w, G.eloc, G.stats, B, G.n, G.na, G.nb, G.h[L + 1], G.d0);
  else
    hipLaunchKernelGGL(k_softmax_bwd<2>, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, G.x, G.w, G.eloc, G.stats, B, G.n, G.na, G.nb, G.h[L + 1], G.d0);
  // backward: d0 holds dz of layer l's output ([B][out]); weights get dz^T h[l]
  double* dcur = G.d0;
  double* dnext = G.d1;
  for (int l = L; l >= 0; --l) {
    const int in = G.dims[l], out = G.dims[l + 1];
    // dW[l][o][k] = sum_b dz[b][o] h[l][b][k]
    gemm(out, in, (int)B, dcur, 1, out, G.h[l], in, 1, G.dW[l], in, nullptr, 0, G.splits, G.part, st);
    // db[l][o] = sum_b dz[b][o]
    gemm(1, out, (int)B, G.ones, 0, 1, dcur, out, 1, G.db[l], out, nullptr, 0, G.splits, G.part, st);
    if (l > 0) {
      // dh[b][k] = sum_o dz[b][o] Wm[l][o][k], then ReLU' of layer l-1's output
      gemm((int)B, in, out, dcur, out, 1, G.Wm[l], in, 1, dnext, in, nullptr, 0, 1, nullptr, st);
      const int64_t cnt = B * in;
      hipLaunchKernelGGL(k_relu_bwd, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, dnext, G.h[l], cnt);
      double* t = dcur; dcur = dnext; dnext = t;
    }
  }
  hipLaunchKernelGGL(k_write_dtheta, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, st, G);
  return hipGetLastError();
}

}  // namespace elocal
