// Autoregressive ansatz on BF16 matrix cores (v_mfma_f32_16x16x32_bf16) and the fused
// local-energy kernel built on it.
//
// Formulation: every layer is computed transposed, D[unit][row] = W[unit][k] * act[k][row],
// so the weights are the A operand and the activations of 16 rows the B operand. The
// 16x16 result gives lane (g = lane/16, r = lane%16) the units 4g..4g+3 of its 16-unit
// block for row r; two such blocks are exactly the 8 k-values lane group g must supply
// as the B operand of the next layer, provided the packed weights of the next layer
// use the matching k order. So activations never leave registers between layers.
// In the output layer the four logits of orbital 4*block + g land in one lane, so the
// number-conserving log-softmax is lane-local.
//
// Precision: layer-0 inputs are exact 0/1; every later activation a (FP32 after bias
// and ReLU) is fed as hi = bf16(a) plus lo = bf16(a - hi), two MFMAs per weight
// fragment, so the representation error is ~2^-18 |a|. Accumulation is FP32; the
// ratio exp(dA + i dphi), the matrix element and every sum are FP64.
#include "elocal_internal.hpp"
#include "kernels.hpp"

namespace elocal {

__device__ __forceinline__ bool made_allowed(int n, int L, int l, int o, int k) {
  const int nm1 = n - 1;
  if (l == 0) return (o % nm1) + 1 >= k / 2 + 1;
  if (l < L) return (o % nm1) + 1 >= (k % nm1) + 1;
  if (o == 4 * n) return true;              // phase head sees the whole last layer
  return (o / 4) + 1 > (k % nm1) + 1;
}

// k index (within a layer's input) of k-slot j of lane group g in k-block kb.
__device__ __forceinline__ int kslot_bf16(int l, int kb, int g, int j) {
  if (l == 0) return 32 * kb + 8 * g + j;
  return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

__global__ void k_pack_bf16(MadeDev M, ThetaLayout T, const uint16_t* __restrict__ theta,
                            bf16x8* __restrict__ frag, float* __restrict__ bias) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nlane = M.nfrag * 64u;
  if (gid < nlane) {
    const uint32_t f = gid >> 6;
    const int lane = gid & 63;
    int l = 0;
    while (l < M.L && f >= M.woff[l + 1]) ++l;
    const uint32_t local = f - M.woff[l];
    const int ob = local / M.nk[l], kb = local % M.nk[l];
    const int o = 16 * ob + (lane & 15), g = lane >> 4;
    unsigned short v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = kslot_bf16(l, kb, g, j);
      unsigned short bits = 0;
      if (o < M.nout[l] && k < M.nin[l] && made_allowed(M.n, M.L, l, o, k)) {
        if (l == M.L && o == 4 * M.n) bits = theta[T.offwphi + k];
        else bits = theta[T.offW[l] + (uint32_t)o * M.nin[l] + k];
      }
      v[j] = bits;
    }
    bf16x8 out;
    __builtin_memcpy(&out, v, sizeof(out));
    frag[gid] = out;
  }
  if (gid < M.nbias) {
    int l = 0;
    while (l < M.L && gid >= M.boff[l + 1]) ++l;
    const int o = gid - M.boff[l];
    unsigned short bits = 0;
    if (o < M.nout[l]) bits = (l == M.L && o == 4 * M.n) ? theta[T.offbphi] : theta[T.offb[l] + o];
    bias[gid] = __uint_as_float((uint32_t)bits << 16);
  }
}

__device__ __forceinline__ bf16x8 bits_to_bf16x8(uint32_t v) {
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    w[q] = (((v >> (2 * q)) & 1u) * 0x3F80u) | ((((v >> (2 * q + 1)) & 1u) * 0x3F80u) << 16);
  bf16x8 r;
  __builtin_memcpy(&r, w, sizeof(r));
  return r;
}

template <int NW>
__device__ __forceinline__ uint32_t byte_at(const uint64_t (&x)[NW], int bit) {
  uint32_t v = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w)
    if ((bit >> 6) == w) v = (uint32_t)((x[w] >> (bit & 63)) & 0xFFull);
  return v;
}

__device__ __forceinline__ void split_relu(const f32x4& a, const f32x4& b, bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float u = fmaxf(a[i], 0.f), v = fmaxf(b[i], 0.f);
    const __bf16 uh = (__bf16)u, vh = (__bf16)v;
    hi[i] = uh; hi[4 + i] = vh;
    lo[i] = (__bf16)(u - (float)uh);
    lo[4 + i] = (__bf16)(v - (float)vh);
  }
}

__device__ __forceinline__ f32x4 mfma_bf16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 load_bias4(const float* bias, uint32_t off) {
  f32x4 r;
  r[0] = bias[off]; r[1] = bias[off + 1]; r[2] = bias[off + 2]; r[3] = bias[off + 3];
  return r;
}

// Runs the network on two 16-row column blocks (rows r and 16 + r of lane r) and calls
// epi(ob, acc_c0, acc_c1) for every 16-unit block of the output layer.
template <int HMAX, int NW, class Epi>
__device__ __forceinline__ void mlp_bf16(const MadeDev& M, const bf16x8* __restrict__ W,
                                         const float* __restrict__ bias,
                                         const uint64_t (&xr)[2][NW], int lane, Epi&& epi) {
  constexpr int KB = HMAX / 32;
  const int g = lane >> 4;
  bf16x8 chi[2][KB], clo[2][KB];
  // ---- layer 0: exact 0/1 inputs, one MFMA per fragment
  {
    const int nk = M.nk[0], nob = M.nob[0];
    bf16x8 xin[2][4];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        xin[c][kb] = bits_to_bf16x8(kb < nk ? byte_at<NW>(xr[c], 32 * kb + 8 * g) : 0u);
#pragma unroll
    for (int kbo = 0; kbo < KB; ++kbo) {
      if (2 * kbo < nob) {
        f32x4 a0[2], a1[2];
        const f32x4 b0 = load_bias4(bias, M.boff[0] + 32 * kbo + 4 * g);
        const f32x4 b1 = load_bias4(bias, M.boff[0] + 32 * kbo + 16 + 4 * g);
        a0[0] = a0[1] = b0; a1[0] = a1[1] = b1;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          if (kb < nk) {
            const bf16x8 w0 = W[(M.woff[0] + (2 * kbo) * nk + kb) * 64 + lane];
            const bf16x8 w1 = W[(M.woff[0] + (2 * kbo + 1) * nk + kb) * 64 + lane];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              a0[c] = mfma_bf16(w0, xin[c][kb], a0[c]);
              a1[c] = mfma_bf16(w1, xin[c][kb], a1[c]);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) split_relu(a0[c], a1[c], chi[c][kbo], clo[c][kbo]);
      }
    }
  }
  // ---- hidden layers 1..L-1: hi + lo activations
  for (int l = 1; l < M.L; ++l) {
    const int nk = M.nk[l], nob = M.nob[l];
    bf16x8 nhi[2][KB], nlo[2][KB];
#pragma unroll
    for (int kbo = 0; kbo < KB; ++kbo) {
      if (2 * kbo < nob) {
        f32x4 a0[2], a1[2];
        const f32x4 b0 = load_bias4(bias, M.boff[l] + 32 * kbo + 4 * g);
        const f32x4 b1 = load_bias4(bias, M.boff[l] + 32 * kbo + 16 + 4 * g);
        a0[0] = a0[1] = b0; a1[0] = a1[1] = b1;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          if (kb < nk) {
            const bf16x8 w0 = W[(M.woff[l] + (2 * kbo) * nk + kb) * 64 + lane];
            const bf16x8 w1 = W[(M.woff[l] + (2 * kbo + 1) * nk + kb) * 64 + lane];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
              a0[c] = mfma_bf16(w0, chi[c][kb], a0[c]);
              a0[c] = mfma_bf16(w0, clo[c][kb], a0[c]);
              a1[c] = mfma_bf16(w1, chi[c][kb], a1[c]);
              a1[c] = mfma_bf16(w1, clo[c][kb], a1[c]);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) split_relu(a0[c], a1[c], nhi[c][kbo], nlo[c][kbo]);
      }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) { chi[c][kb] = nhi[c][kb]; clo[c][kb] = nlo[c][kb]; }
  }
  // ---- output layer: 4n logits + phase row, block by block into the epilogue
  {
    const int l = M.L, nk = M.nk[l], nob = M.nob[l];
#pragma unroll 1
    for (int ob = 0; ob < nob; ++ob) {
      f32x4 a[2];
      a[0] = a[1] = load_bias4(bias, M.boff[l] + 16 * ob + 4 * g);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        if (kb < nk) {
          const bf16x8 w = W[(M.woff[l] + ob * nk + kb) * 64 + lane];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            a[c] = mfma_bf16(w, chi[c][kb], a[c]);
            a[c] = mfma_bf16(w, clo[c][kb], a[c]);
          }
        }
      }
      epi(ob, a[0], a[1]);
    }
  }
}

// log p_p(s) of the occupation s of orbital p in row x (FP32 log-softmax over the
// occupations that keep both electron counts reachable).
template <int NW>
__device__ __forceinline__ float cond_logp(const uint64_t (&x)[NW], int p, int n, int na, int nb,
                                           const f32x4& z) {
  const int cu = count_spin_below<NW>(x, p, 0), cd = count_spin_below<NW>(x, p, 1);
  const int left = n - p - 1;
  const int s = getbit<NW>(x, 2 * p) + 2 * getbit<NW>(x, 2 * p + 1);
  bool ok[4];
  float m = -INFINITY;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = cu + (q & 1), d = cd + (q >> 1);
    ok[q] = (u <= na) && (d <= nb) && (u + left >= na) && (d + left >= nb);
    if (ok[q]) m = fmaxf(m, z[q]);
  }
  float sum = 0.f;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (ok[q]) sum += __expf(z[q] - m);
  const float zs = (s == 0) ? z[0] : (s == 1) ? z[1] : (s == 2) ? z[2] : z[3];
  return zs - m - __logf(sum);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------------------------- sample pass
// A(x), phi(x) and the per-orbital log p_p(s_p) of every sample (32 samples per wave step).
template <int HMAX, int NW>
__global__ void __launch_bounds__(256) k_rows_bf16(RowsArgs P) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t b0 = wave * 32;
  if (b0 >= P.B) return;
  const MadeDev& M = P.made;
  const int n = P.sys.n, na = P.sys.na, nb = P.sys.nb;
  const bf16x8* W = (const bf16x8*)M.wfrag;
  const float* bias = (const float*)M.bias;
  uint64_t xr[2][NW];
  int64_t rb[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    rb[c] = b0 + 16 * c + r16;
    const int64_t bb = rb[c] < P.B ? rb[c] : b0;
#pragma unroll
    for (int w = 0; w < NW; ++w) xr[c][w] = P.x[bb * NW + w];
  }
  const int ob_phi = (4 * n) >> 4, g_phi = ((4 * n) & 15) >> 2;
  double A[2] = {0.0, 0.0};
  float zp[2] = {0.f, 0.f};
  mlp_bf16<HMAX, NW>(M, W, bias, xr, lane, [&](int ob, const f32x4& a0, const f32x4& a1) {
    const int p = 4 * ob + g;
    if (p < n) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float lp = cond_logp<NW>(xr[c], p, n, na, nb, c ? a1 : a0);
        A[c] += (double)lp;
        if (rb[c] < P.B) P.lpx[rb[c] * n + p] = lp;
      }
    }
    if (ob == ob_phi && g == g_phi) { zp[0] = a0[0]; zp[1] = a1[0]; }
  });
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    A[c] += __shfl_xor(A[c], 16);
    A[c] += __shfl_xor(A[c], 32);
    zp[c] = __shfl(zp[c], g_phi * 16 + r16);
  }
  if (g < 2) {
    const int c = g;
    if (rb[c] < P.B) {
      P.zphi[rb[c]] = (double)zp[c];
      if (P.logpsi) {
        const double sig = 1.0 / (1.0 + exp(-(double)zp[c]));
        P.logpsi[2 * rb[c]] = 0.5 * A[c];
        P.logpsi[2 * rb[c] + 1] = 2.0 * M_PI * sig;
      }
    }
  }
}

// ----------------------------------------------------------------------------- fused eval
struct WaveCtxBF16 {
  SampleCtx c;
  float lpx[kMaxOrb];
};

template <int HMAX, int NW, bool LDSW>
__global__ void __launch_bounds__(256) k_eval_bf16(EvalArgs P) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, g = lane >> 4, r16 = lane & 15;
  const MadeDev& M = P.made;
  const SysDev& S = P.sys;
  const bf16x8* W = (const bf16x8*)M.wfrag;
  const float* bias = (const float*)M.bias;
  if (LDSW) {
    bf16x8* sw = (bf16x8*)smem;
    const bf16x8* gw = (const bf16x8*)M.wfrag;
    for (uint32_t i = threadIdx.x; i < M.nfrag * 64u; i += blockDim.x) sw[i] = gw[i];
    float* sb = (float*)(smem + P.lds_bias_off);
    for (uint32_t i = threadIdx.x; i < M.nbias; i += blockDim.x) sb[i] = bias[i];
    __syncthreads();
    W = sw;
    bias = sb;
  }
  WaveCtxBF16& wc = ((WaveCtxBF16*)(smem + P.lds_ctx_off))[wid];
  const int n = S.n, na = S.na, nb = S.nb;
  const int ob_phi = (4 * n) >> 4, g_phi = ((4 * n) & 15) >> 2;
  const uint32_t nS = S.nSa + S.nSb;
  int64_t cur_b = -1;
  uint64_t xs[NW];
  double sig_x = 0.0, ed = 0.0;
  const double* Fs = P.F;
  for (int64_t item = (int64_t)blockIdx.x * 4 + wid; item < P.n_items; item += (int64_t)gridDim.x * 4) {
    const int64_t b = item / P.ips;
    const uint32_t seg = (uint32_t)(item % P.ips);
    if (b != cur_b) {
      wave_sync_lds();
#pragma unroll
      for (int w = 0; w < NW; ++w) xs[w] = P.x[b * NW + w];
      build_ctx<NW>(S, xs, wc.c, lane);
      if (lane < n) wc.lpx[lane] = P.lpx[b * n + lane];
      wave_sync_lds();
      sig_x = 1.0 / (1.0 + exp(-P.zphi[b]));
      ed = P.ediag[b];
      Fs = P.F + (size_t)b * nS;
      cur_b = b;
    }
    double acc_re = 0.0, acc_im = 0.0;
    for (uint32_t tile = 0; tile < P.tpi; ++tile) {
      const uint32_t t0 = 1u + (seg * P.tpi + tile) * 32u;
      if (t0 >= S.C) break;
      const uint32_t t = t0 + (lane & 31);
      uint64_t xp[NW];
      double hv = 0.0;
      if (t < S.C) {
        const Excitation e = unrank(S, wc.c, t);
        const int sg = apply_excitation<NW>(xs, e, xp);
        if (lane < 32) {
          const double v = excitation_value(S, e, Fs, ed);
          hv = sg < 0 ? -v : v;
        }
      } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) xp[w] = xs[w];
      }
      uint64_t xr[2][NW];
      const bool own1 = (lane >> 4) & 1;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint64_t other = __shfl_xor(xp[w], 16);
        xr[0][w] = own1 ? other : xp[w];
        xr[1][w] = own1 ? xp[w] : other;
      }
      const int p0[2] = {first_diff_orbital<NW>(xs, xr[0], n), first_diff_orbital<NW>(xs, xr[1], n)};
      double dA[2] = {0.0, 0.0};
      float zp[2] = {0.f, 0.f};
      mlp_bf16<HMAX, NW>(M, W, bias, xr, lane, [&](int ob, const f32x4& a0, const f32x4& a1) {
        const int p = 4 * ob + g;
        if (p < n) {
          const float lx = wc.lpx[p];
#pragma unroll
          for (int c = 0; c < 2; ++c)
            if (p >= p0[c]) dA[c] += (double)(cond_logp<NW>(xr[c], p, n, na, nb, c ? a1 : a0) - lx);
        }
        if (ob == ob_phi && g == g_phi) { zp[0] = a0[0]; zp[1] = a1[0]; }
      });
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        dA[c] += __shfl_xor(dA[c], 16);
        dA[c] += __shfl_xor(dA[c], 32);
        zp[c] = __shfl(zp[c], g_phi * 16 + r16);
      }
      if (lane < 32) {
        const int c = lane >> 4;
        const double da = 0.5 * (c ? dA[1] : dA[0]);
        const double z = (double)(c ? zp[1] : zp[0]);
        const double dphi = 2.0 * M_PI * (1.0 / (1.0 + exp(-z)) - sig_x);
        double sn, cs;
        sincos(dphi, &sn, &cs);
        const double mag = hv * exp(da);
        acc_re += mag * cs;
        acc_im += mag * sn;
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      acc_re += __shfl_xor(acc_re, off);
      acc_im += __shfl_xor(acc_im, off);
    }
    if (lane == 0) {
      P.partial[2 * item] = acc_re;
      P.partial[2 * item + 1] = acc_im;
    }
  }
}

// ----------------------------------------------------------------------------- launchers
hipError_t launch_pack_bf16(const MadeDev& M, const ThetaLayout& T, const uint16_t* theta,
                            void* frag, float* bias, hipStream_t st) {
  const uint32_t total = M.nfrag * 64u > M.nbias ? M.nfrag * 64u : M.nbias;
  hipLaunchKernelGGL(k_pack_bf16, dim3((total + 255) / 256), dim3(256), 0, st, M, T, theta,
                     (bf16x8*)frag, bias);
  return hipGetLastError();
}

template <int HMAX>
static hipError_t rows_bf16_h(const RowsArgs& A, hipStream_t st) {
  const int64_t waves = (A.B + 31) / 32;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  if (A.sys.W == 1) hipLaunchKernelGGL((k_rows_bf16<HMAX, 1>), dim3(blocks), dim3(256), 0, st, A);
  else hipLaunchKernelGGL((k_rows_bf16<HMAX, 2>), dim3(blocks), dim3(256), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_rows_bf16(const RowsArgs& A, int hmax, hipStream_t st) {
  if (A.B <= 0) return hipSuccess;
  switch (hmax) {
    case 32: return rows_bf16_h<32>(A, st);
    case 64: return rows_bf16_h<64>(A, st);
    case 128: return rows_bf16_h<128>(A, st);
    case 256: return rows_bf16_h<256>(A, st);
  }
  return hipErrorInvalidValue;
}

template <int HMAX, int NW, bool LDSW>
static hipError_t eval_bf16_k(const EvalArgs& A, size_t lds, unsigned grid, hipStream_t st) {
  auto kern = k_eval_bf16<HMAX, NW, LDSW>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(256), lds, st, A);
  return hipGetLastError();
}

template <int HMAX>
static hipError_t eval_bf16_h(const EvalArgs& A, bool ldsw, size_t lds, unsigned grid, hipStream_t st) {
  if (A.sys.W == 1)
    return ldsw ? eval_bf16_k<HMAX, 1, true>(A, lds, grid, st) : eval_bf16_k<HMAX, 1, false>(A, lds, grid, st);
  return ldsw ? eval_bf16_k<HMAX, 2, true>(A, lds, grid, st) : eval_bf16_k<HMAX, 2, false>(A, lds, grid, st);
}

hipError_t launch_eval_bf16(const EvalArgs& A, int hmax, bool ldsw, size_t lds, unsigned grid,
                            hipStream_t st) {
  if (A.n_items <= 0) return hipSuccess;
  switch (hmax) {
    case 32: return eval_bf16_h<32>(A, ldsw, lds, grid, st);
    case 64: return eval_bf16_h<64>(A, ldsw, lds, grid, st);
    case 128: return eval_bf16_h<128>(A, ldsw, lds, grid, st);
    case 256: return eval_bf16_h<256>(A, ldsw, lds, grid, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace elocal
