// Autoregressive ansatz on FP64 matrix cores (v_mfma_f64_16x16x4f64) and the fused
// all-FP64 local-energy kernel.
//
// Same transposed formulation as the BF16 path (weights = A operand, 16 rows = B
// operand). The FP64 instruction returns row 4*i + lane/16 of the 16x16 block in
// register i, so the packer stores weight row 16*ob + 4*(rho%4) + rho/4 at A-row rho;
// lane group g then holds units 16*ob + 4g + i in register i, exactly as in the BF16
// path, and register i of block ob is the B operand of k-step 4*ob + i of the next
// layer. Output orbital 4*ob + g again lands in one lane. Hidden units are stored in
// degree order, so o-block ob of layer l only needs its first kend[l][ob] k-steps (whole
// 16-unit blocks of the previous layer; the rest of its weights are masked).
#include "elocal_internal.hpp"
#include "kernels.hpp"

namespace elocal {

__device__ __forceinline__ bool made_allowed64(int n, int L, int l, int o, int k) {
  const int nm1 = n - 1;
  if (l == 0) return (o % nm1) + 1 >= k / 2 + 1;
  if (l < L) return (o % nm1) + 1 >= (k % nm1) + 1;
  if (o == 4 * n) return true;
  return (o / 4) + 1 > (k % nm1) + 1;
}

__global__ void k_pack_f64(MadeDev M, ThetaLayout T, const double* __restrict__ theta,
                           double* __restrict__ frag, double* __restrict__ bias) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid < M.nfrag * 64u) {
    const uint32_t f = gid >> 6;
    const int lane = gid & 63;
    int l = 0;
    while (l < M.L && f >= M.woff[l + 1]) ++l;
    const uint32_t local = f - M.woff[l];
    const int ob = local / M.nk[l], ks = local % M.nk[l];
    const int rho = lane & 15, g = lane >> 4;
    const int opos = 16 * ob + 4 * (rho & 3) + (rho >> 2);
    const int kpos = (l == 0) ? 4 * ks + g : 16 * (ks >> 2) + 4 * g + (ks & 3);
    // hidden units in degree order (as in the BF16 packing); inputs and logits unsorted
    const int o = (l < M.L && opos < M.nout[l]) ? sorted_unit(M.n, M.nout[l], opos) : opos;
    const int k = (l > 0 && kpos < M.nin[l]) ? sorted_unit(M.n, M.nin[l], kpos) : kpos;
    double v = 0.0;
    if (o < M.nout[l] && k < M.nin[l] && made_allowed64(M.n, M.L, l, o, k)) {
      if (l == M.L && o == 4 * M.n) v = theta[T.offwphi + k];
      else v = theta[T.offW[l] + (uint32_t)o * M.nin[l] + k];
    }
    frag[gid] = v;
  }
  if (gid < M.nbias) {
    int l = 0;
    while (l < M.L && gid >= M.boff[l + 1]) ++l;
    const int opos = gid - M.boff[l];
    double v = 0.0;
    if (opos < M.nout[l]) {
      const int o = (l < M.L) ? sorted_unit(M.n, M.nout[l], opos) : opos;
      v = (l == M.L && o == 4 * M.n) ? theta[T.offbphi] : theta[T.offb[l] + o];
    }
    bias[gid] = v;
  }
}

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, const f64x4& c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f64x4 relu4(const f64x4& a) {
  f64x4 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) r[i] = a[i] > 0.0 ? a[i] : 0.0;
  return r;
}

// Weight loads of the FP64 network. From global memory through a buffer resource: the
// lane's byte offset stays in one VGPR and the fragment's offset is a scalar, so the
// unrolled k-loops keep no 64-bit address per k-step live (with two waves per SIMD those
// addresses alone would not fit); a load past the packed buffer returns zero.
struct WGlobal64 {
  __amdgpu_buffer_rsrc_t r;
  uint32_t voff;    // lane * 8
  uint32_t frag0;   // the o-block's first fragment
  __device__ __forceinline__ double operator()(int ks) const {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, (frag0 + (uint32_t)ks) * 512u, 0);
    double d;
    __builtin_memcpy(&d, &v, 8);
    return d;
  }
};
// From LDS (or any pointer): fragment ks of the o-block at p (p includes the lane).
struct WPtr64 {
  const double* p;
  __device__ __forceinline__ double operator()(int ks) const { return p[ks * 64]; }
};
// Biases of rows 4g..4g+3 of the 16-row block starting at padded bias `blk`: two 16-byte
// loads with the lane's offset in a VGPR and the block's as a scalar.
__device__ __forceinline__ f64x4 bias4_rsrc(const __amdgpu_buffer_rsrc_t& r, uint32_t voff_g, uint32_t blk) {
  const auto lo = __builtin_amdgcn_raw_buffer_load_b128(r, voff_g, blk * 8u, 0);
  const auto hi = __builtin_amdgcn_raw_buffer_load_b128(r, voff_g + 16u, blk * 8u, 0);
  double d[4];
  __builtin_memcpy(d, &lo, 16);
  __builtin_memcpy(d + 2, &hi, 16);
  return f64x4{d[0], d[1], d[2], d[3]};
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t bias_rsrc64(const MadeDev& M) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(M.bias), (short)0, (int)(M.nbias * 8u), 0x00020000);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t weight_rsrc64(const MadeDev& M) {
  // word 3 = 0x00020000: raw (untyped) buffer access on the gfx9 family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(M.wfrag), (short)0, (int)(M.nfrag * 512u), 0x00020000);
}

// k-steps [0, ke) of one o-block: f(ks, w) with w = ld(ks), the weight loads running
// two chunks of CH k-steps ahead of the products that use them (one wave per SIMD has
// nothing else to hide the load latency with). CH = 8 measured best at width <= 128;
// width 256 keeps CH = 4 (fewer registers).
template <int KSMAX, int CH, class Ld, class F>
__device__ __forceinline__ void kloop_f64(const Ld& ld, int ke, F&& f) {
  constexpr int LA = 2, NC = (KSMAX + CH - 1) / CH;
  double w[NC][CH];
#pragma unroll
  for (int c = 0; c < LA && c < NC; ++c)
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if (c * CH + j < ke) w[c][j] = ld(c * CH + j);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    // keeps the scheduler from hoisting later chunks' loads (their registers) above this point
    __builtin_amdgcn_sched_barrier(0);
    if (c * CH < ke) {
      if (c + LA < NC) {
#pragma unroll
        for (int j = 0; j < CH; ++j)
          if ((c + LA) * CH + j < ke) w[c + LA][j] = ld((c + LA) * CH + j);
      }
#pragma unroll
      for (int j = 0; j < CH; ++j)
        if (c * CH + j < ke) f(c * CH + j, w[c][j]);
    }
  }
}

// As kloop_f64 for a block whose k-range is whole chunks (ke a multiple of CH, at most the
// block's stored k-steps): one branch per chunk instead of one per k-step.
template <int KSMAX, int CH, class Ld, class F>
__device__ __forceinline__ void kloop_f64_whole(const Ld& ld, int ke, F&& f) {
  constexpr int LA = 2, NC = (KSMAX + CH - 1) / CH;
  double w[NC][CH];
#pragma unroll
  for (int c = 0; c < LA && c < NC; ++c)
    if (c * CH < ke) {
#pragma unroll
      for (int j = 0; j < CH; ++j) w[c][j] = ld(c * CH + j);
    }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    __builtin_amdgcn_sched_barrier(0);
    if (c * CH < ke) {
      if (c + LA < NC && (c + LA) * CH < ke) {
#pragma unroll
        for (int j = 0; j < CH; ++j) w[c + LA][j] = ld((c + LA) * CH + j);
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) f(c * CH + j, w[c][j]);
    }
  }
}

// Hidden blocks to compute per layer (with CAP): the rest are set to zero.
struct HiddenCaps {
  int nob[kMaxLayers];
};

// Network on one 16-row block (row r of lane r); epi(ob, acc) per output block ob in
// [ob_lo, ob_hi) (all of them by default). Weights come from the packed buffer M.wfrag
// (layer l at fragment woff[l]); with OUT_LDS the output layer's come from WL, a copy of its
// fragments in LDS. With CAP only the first
// caps.nob[l] blocks of hidden layer l are computed and the others are zero (a block the
// caller needs must not depend on the skipped ones).
//
// With INPLACE the hidden layers keep one activation array: output blocks are computed from
// the highest down, and block ob + 1's result waits in a register set until block ob has
// read its inputs; it then overwrites input block ob + 1, which no lower block reads. Exact
// when every block ob of a hidden layer reads input blocks <= ob + 1 (inplace_ok_f64 on the
// host); half the activation registers, so two waves fit per SIMD at widths 128 and 256.
template <int HMAX, int NW, bool CAP = false, bool INPLACE = false, bool OUT_LDS = false, class Epi>
__device__ __forceinline__ void mlp_f64(const MadeDev& M, const double* __restrict__ WL,
                                        const uint64_t (&xr)[NW], int lane, Epi&& epi, int ob_lo = 0,
                                        int ob_hi = kMaxOutBlocks, const HiddenCaps& caps = HiddenCaps{}) {
  static_assert(!(CAP && INPLACE), "capped layers are computed out of place");
  constexpr int OB = HMAX / 16;
  constexpr int KS = HMAX / 4;
  // k-steps per weight-load chunk (the in-place variant's row of chunks is what its
  // exactness condition assumes)
  constexpr int KCH = (HMAX >= 256 || INPLACE) ? 4 : 8;
  const int g = lane >> 4;
  const __amdgpu_buffer_rsrc_t rs = weight_rsrc64(M), rb = bias_rsrc64(M);
  const uint32_t voff = (uint32_t)lane * 8u, voff_g = (uint32_t)g * 32u;
  f64x4 cur[OB];
  {
    const int nk = M.nk[0], nob = CAP ? min(M.nob[0], caps.nob[0]) : M.nob[0];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      if (CAP && ob >= nob) cur[ob] = f64x4{0.0, 0.0, 0.0, 0.0};
      if (ob < nob) {
        const int ke = __builtin_amdgcn_readfirstlane(M.kend[0][ob]);
        f64x4 acc = bias4_rsrc(rb, voff_g, M.boff[0] + 16 * ob);
        const WGlobal64 wl{rs, voff, M.woff[0] + (uint32_t)(ob * nk)};
        if constexpr (NW == 1 && HMAX <= 128) {
          // one-word determinants (2n <= 64 bits, at most 16 k-steps): loads run ahead
          kloop_f64<16, 4>(wl, ke, [&](int ks, double w) {
            acc = mfma_f64(w, (double)getbit<NW>(xr, 4 * ks + g), acc);
          });
        } else {
          // longer inputs or wider networks: the registers for prefetching are not there
          for (int ks = 0; ks < ke; ++ks) {
            const double bv = (double)getbit<NW>(xr, 4 * ks + g);
            acc = mfma_f64(wl(ks), bv, acc);
          }
        }
        cur[ob] = relu4(acc);
      }
    }
  }
  for (int l = 1; l < M.L && INPLACE; ++l) {
    const int nk = M.nk[l], nob = M.nob[l];
    f64x4 pend = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ob = OB - 1; ob >= 0; --ob) {
      if (ob < nob) {
        const int ke = __builtin_amdgcn_readfirstlane(M.kend[l][ob]);
        f64x4 acc = bias4_rsrc(rb, voff_g, M.boff[l] + 16 * ob);
        const WGlobal64 wl{rs, voff, M.woff[l] + (uint32_t)(ob * nk)};
        const int kw = min(nk, (ke + KCH - 1) / KCH * KCH);
        kloop_f64_whole<KS, KCH>(wl, kw, [&](int ks, double w) { acc = mfma_f64(w, cur[ks >> 2][ks & 3], acc); });
        if (ob + 1 < nob) cur[ob + 1] = pend;
        pend = relu4(acc);
      }
    }
    cur[0] = pend;
  }
  for (int l = 1; l < M.L && !INPLACE; ++l) {
    const int nk = M.nk[l], nob = CAP ? min(M.nob[l], caps.nob[l]) : M.nob[l];
    f64x4 nxt[OB];
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      if (CAP && ob >= nob) nxt[ob] = f64x4{0.0, 0.0, 0.0, 0.0};
      if (ob < nob) {
        const int ke = __builtin_amdgcn_readfirstlane(M.kend[l][ob]);
        f64x4 acc = bias4_rsrc(rb, voff_g, M.boff[l] + 16 * ob);
        const WGlobal64 wl{rs, voff, M.woff[l] + (uint32_t)(ob * nk)};
        // whole chunks: the extra k-steps up to a chunk boundary hold masked (zero) weights,
        // and nk (width / 4, widths are multiples of 32) is a multiple of the chunk
        const int kw = min(nk, (ke + KCH - 1) / KCH * KCH);
        kloop_f64_whole<KS, KCH>(wl, kw, [&](int ks, double w) { acc = mfma_f64(w, cur[ks >> 2][ks & 3], acc); });
        nxt[ob] = relu4(acc);
      }
    }
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) cur[ob] = nxt[ob];
  }
  {
    const int l = M.L, nk = M.nk[l], nob = min(M.nob[l], ob_hi);
#pragma unroll 1
    for (int ob = ob_lo; ob < nob; ++ob) {
      const int ke = __builtin_amdgcn_readfirstlane(M.kend[l][ob]);
      f64x4 acc = bias4_rsrc(rb, voff_g, M.boff[l] + 16 * ob);
      const int kw = min(nk, (ke + KCH - 1) / KCH * KCH);   // whole chunks, as above
      auto step = [&](int ks, double w) { acc = mfma_f64(w, cur[ks >> 2][ks & 3], acc); };
      if constexpr (OUT_LDS) kloop_f64_whole<KS, KCH>(WPtr64{WL + (size_t)(ob * nk) * 64 + lane}, kw, step);
      else kloop_f64_whole<KS, KCH>(WGlobal64{rs, voff, M.woff[l] + (uint32_t)(ob * nk)}, kw, step);
      epi(ob, acc);
    }
  }
}

template <int NW>
__device__ __forceinline__ double cond_logp64(const uint64_t (&x)[NW], int p, int n, int na, int nb,
                                              const f64x4& z) {
  const int cu = count_spin_below<NW>(x, p, 0), cd = count_spin_below<NW>(x, p, 1);
  const int left = n - p - 1;
  const int s = getbit<NW>(x, 2 * p) + 2 * getbit<NW>(x, 2 * p + 1);
  bool ok[4];
  double m = -INFINITY;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = cu + (q & 1), d = cd + (q >> 1);
    ok[q] = (u <= na) && (d <= nb) && (u + left >= na) && (d + left >= nb);
    if (ok[q]) m = fmax(m, z[q]);
  }
  double sum = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (ok[q]) sum += exp(z[q] - m);
  const double zs = (s == 0) ? z[0] : (s == 1) ? z[1] : (s == 2) ? z[2] : z[3];
  return zs - m - log(sum);
}

__device__ __forceinline__ void wave_sync_lds64() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int HMAX, int NW>
__global__ void __launch_bounds__(256) k_rows_f64(RowsArgs P) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t b0 = wave * 16;
  const int64_t Bn = P.count ? min(P.B, *P.count) : P.B;
  if (b0 >= Bn) return;
  const MadeDev& M = P.made;
  const int n = P.sys.n, na = P.sys.na, nb = P.sys.nb;
  const int64_t rb = b0 + r16;
  const int64_t bb = rb < Bn ? rb : b0;
  uint64_t xr[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) xr[w] = P.x[bb * NW + w];
  const int ob_phi = (4 * n) >> 4, g_phi = ((4 * n) & 15) >> 2;
  double A = 0.0, zp = 0.0;
  mlp_f64<HMAX, NW>(M, nullptr, xr, lane,
                    [&](int ob, const f64x4& a) {
                      const int p = 4 * ob + g;
                      if (p < n) {
                        const double lp = cond_logp64<NW>(xr, p, n, na, nb, a);
                        A += lp;
                        if (rb < Bn) P.lpx64[rb * n + p] = lp;
                      }
                      if (ob == ob_phi && g == g_phi) zp = a[0];
                    });
  A += __shfl_xor(A, 16);
  A += __shfl_xor(A, 32);
  zp = __shfl(zp, g_phi * 16 + r16);
  if (g == 0 && rb < Bn) {
    P.zphi[rb] = zp;
    if (P.logpsi) {
      P.logpsi[2 * rb] = 0.5 * A;
      P.logpsi[2 * rb + 1] = 2.0 * M_PI / (1.0 + exp(-zp));
    }
  }
}

struct WaveCtx64 {
  SampleCtx c;
  double lpx[kMaxOrb];
};

template <int NW>
struct SampleState64 {
  int64_t b;
  uint64_t xs[NW];
  double sig_x, ed;
  const double* Fs;
};

// One work item = one sample and P.tpi tiles of 16 list entries; the 64 lanes of a tile
// share its 16 rows (lane group g holds output units 4g..4g+3 of each 16-unit block).
template <int HMAX, int NW, bool INPLACE = false, bool OUT_LDS = false>
__device__ __forceinline__ void eval_item_f64(const EvalArgs& P, const double* __restrict__ WL, WaveCtx64& wc,
                                              int64_t item, SampleState64<NW>& st, int lane) {
  const MadeDev& M = P.made;
  const SysDev& S = P.sys;
  const int g = lane >> 4, r16 = lane & 15;
  const int n = S.n, na = S.na, nb = S.nb;
  const int ob_phi = (4 * n) >> 4, g_phi = ((4 * n) & 15) >> 2;
  const int64_t b = item / P.ips;
  const uint32_t seg = (uint32_t)(item % P.ips);
  if (b != st.b) {
    wave_sync_lds64();
#pragma unroll
    for (int w = 0; w < NW; ++w) st.xs[w] = P.x[b * NW + w];
    build_ctx<NW>(S, st.xs, wc.c, lane);
    if (lane < n) wc.lpx[lane] = P.lpx64[b * n + lane];
    wave_sync_lds64();
    st.sig_x = 1.0 / (1.0 + exp(-P.zphi[b]));
    st.ed = P.ediag[b];
    st.Fs = P.F + (size_t)b * (S.nSa + S.nSb);
    st.b = b;
  }
  const uint64_t(&xs)[NW] = st.xs;
  double acc_re = 0.0, acc_im = 0.0;
  for (uint32_t tile = 0; tile < P.tpi; ++tile) {
    const uint32_t t0 = 1u + (seg * P.tpi + tile) * 16u;
    if (t0 >= S.C) break;
    const uint32_t t = t0 + r16;
    uint64_t xp[NW];
    double hv = 0.0;
    if (t < S.C) {
      const Excitation e = unrank(S, wc.c, t);
      const int sg = apply_excitation<NW>(xs, e, xp);
      if (g == 0) {
        const double v = excitation_value(S, e, st.Fs, st.ed);
        hv = sg < 0 ? -v : v;
      }
    } else {
#pragma unroll
      for (int w = 0; w < NW; ++w) xp[w] = xs[w];
    }
    const int p0 = first_diff_orbital<NW>(xs, xp, n);
    double dA = 0.0, zp = 0.0;
    mlp_f64<HMAX, NW, false, INPLACE, OUT_LDS>(M, WL, xp, lane, [&](int ob, const f64x4& a) {
      const int p = 4 * ob + g;
      if (p < n && p >= p0) dA += cond_logp64<NW>(xp, p, n, na, nb, a) - wc.lpx[p];
      if (ob == ob_phi && g == g_phi) zp = a[0];
    });
    dA += __shfl_xor(dA, 16);
    dA += __shfl_xor(dA, 32);
    zp = __shfl(zp, g_phi * 16 + r16);
    if (g == 0) {
      const double dphi = 2.0 * M_PI * (1.0 / (1.0 + exp(-zp)) - st.sig_x);
      double sn, cs;
      sincos(dphi, &sn, &cs);
      const double mag = hv * exp(0.5 * dA);
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

// With LDSO the output layer's packed weights are first copied to LDS (dynamic shared
// memory of nob[L] * nk[L] fragments). The in-place variant is built for two waves per
// SIMD (256 registers per lane).
template <int HMAX, int NW, bool LDSO, bool INPLACE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(INPLACE ? 2 : 1)))
k_eval_f64(EvalArgs P) {
  __shared__ WaveCtx64 ctxs[4];
  extern __shared__ __attribute__((aligned(16))) double wout[];
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const MadeDev& M = P.made;
  const double* WL = (const double*)M.wfrag + (size_t)M.woff[M.L] * 64;
  if (LDSO) {
    const uint32_t cnt = (uint32_t)(M.nob[M.L] * M.nk[M.L]) * 64u;
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x) wout[i] = WL[i];
    __syncthreads();
    WL = wout;
  }
  SampleState64<NW> st;
  st.b = -1;
  for (int64_t item = (int64_t)blockIdx.x * 4 + wid; item < P.n_items; item += (int64_t)gridDim.x * 4)
    eval_item_f64<HMAX, NW, INPLACE, LDSO>(P, WL, ctxs[wid], item, st, lane);
}

// Several systems in one persistent launch (item index space as in the BF16 kernel).
template <int HMAX>
__global__ void __launch_bounds__(256)
    k_eval_multi_f64(const EvalArgs* __restrict__ args, const int64_t* __restrict__ first, int n_sys) {
  __shared__ WaveCtx64 ctxs[4];
  const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  SampleState64<1> st1;
  SampleState64<2> st2;
  st1.b = st2.b = -1;
  int cur = -1;
  const int64_t total = first[n_sys];
  for (int64_t item = (int64_t)blockIdx.x * 4 + wid; item < total; item += (int64_t)gridDim.x * 4) {
    int s = 0;
    while (s + 1 < n_sys && item >= first[s + 1]) ++s;
    s = __builtin_amdgcn_readfirstlane(s);
    if (s != cur) {
      st1.b = st2.b = -1;
      cur = s;
    }
    const EvalArgs& P = args[s];
    const int64_t local = item - first[s];
    if (P.sys.W == 1) eval_item_f64<HMAX, 1>(P, nullptr, ctxs[wid], local, st1, lane);
    else eval_item_f64<HMAX, 2>(P, nullptr, ctxs[wid], local, st2, lane);
  }
}

// Conditional of orbital k for every prefix: probs[i][s] (0 where s is not reachable).
// FP64 network, 16 prefixes per wave (the layout of the FP64 sample pass).
template <int HMAX, int NW>
__global__ void __launch_bounds__(256) k_bas_probs(SysDev S, MadeDev M, HiddenCaps caps,
                                                   const uint64_t* __restrict__ pre, const int64_t* __restrict__ Ud,
                                                   int64_t cap, int k, double* __restrict__ probs) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t b0 = wave * 16;
  const int64_t U = min(*Ud, cap);
  if (b0 >= U) return;
  const int n = S.n, na = S.na, nb = S.nb;
  const int64_t rb = b0 + r16;
  const int64_t bb = rb < U ? rb : b0;
  uint64_t xr[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) xr[w] = pre[bb * NW + w];
  mlp_f64<HMAX, NW, true>(M, nullptr, xr, lane, [&](int ob, const f64x4& z) {
    if (4 * ob + g != k) return;
    const int cu = count_spin_below<NW>(xr, k, 0), cd = count_spin_below<NW>(xr, k, 1);
    const int left = n - k - 1;
    bool ok[4];
    double m = -INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = cu + (q & 1), d = cd + (q >> 1);
      ok[q] = (u <= na) && (d <= nb) && (u + left >= na) && (d + left >= nb);
      if (ok[q]) m = fmax(m, z[q]);
    }
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (ok[q]) sum += exp(z[q] - m);
    const double lse = m + log(sum);
    if (rb < U) {
#pragma unroll
      for (int q = 0; q < 4; ++q) probs[rb * 4 + q] = ok[q] ? exp(z[q] - lse) : 0.0;
    }
  }, k >> 2, (k >> 2) + 1, caps);   // only orbital k's output block and what it depends on
}

hipError_t launch_pack_f64(const MadeDev& M, const ThetaLayout& T, const double* theta, void* frag,
                           double* bias, hipStream_t st) {
  const uint32_t total = M.nfrag * 64u > M.nbias ? M.nfrag * 64u : M.nbias;
  hipLaunchKernelGGL(k_pack_f64, dim3((total + 255) / 256), dim3(256), 0, st, M, T, theta,
                     (double*)frag, bias);
  return hipGetLastError();
}

template <int HMAX>
static hipError_t rows_f64_h(const RowsArgs& A, hipStream_t st) {
  const int64_t waves = (A.B + 15) / 16;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  if (A.sys.W == 1) hipLaunchKernelGGL((k_rows_f64<HMAX, 1>), dim3(blocks), dim3(256), 0, st, A);
  else hipLaunchKernelGGL((k_rows_f64<HMAX, 2>), dim3(blocks), dim3(256), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_rows_f64(const RowsArgs& A, int hmax, hipStream_t st) {
  if (A.B <= 0) return hipSuccess;
  switch (hmax) {
    case 32: return rows_f64_h<32>(A, st);
    case 64: return rows_f64_h<64>(A, st);
    case 128: return rows_f64_h<128>(A, st);
    case 256: return rows_f64_h<256>(A, st);
  }
  return hipErrorInvalidValue;
}

// Launches k_eval_f64 with the output layer in LDS when it fits beside the kernel's
// static LDS (one 4-wave block per CU; two for the in-place variant, which has half the
// LDS each), else reading it from global memory.
template <int HMAX, int NW, bool INPLACE>
static hipError_t eval_f64_nw(const EvalArgs& A, unsigned grid, hipStream_t st) {
  constexpr size_t kLds = (INPLACE ? 80 : 160) * 1024;
  static size_t static_lds = ~(size_t)0;   // a property of the code object: the same on every device
  if (static_lds == ~(size_t)0) {
    hipFuncAttributes fa;
    const hipError_t e = hipFuncGetAttributes(&fa, (const void*)k_eval_f64<HMAX, NW, true, INPLACE>);
    if (e != hipSuccess) return e;
    static_lds = fa.sharedSizeBytes;
  }
  const size_t out = (size_t)A.made.nob[A.made.L] * A.made.nk[A.made.L] * 64 * sizeof(double);
  if (static_lds + out <= kLds) {
    if (out > 65536) {
      const hipError_t e = hipFuncSetAttribute((const void*)k_eval_f64<HMAX, NW, true, INPLACE>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)out);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_eval_f64<HMAX, NW, true, INPLACE>), dim3(grid), dim3(256), out, st, A);
  } else {
    hipLaunchKernelGGL((k_eval_f64<HMAX, NW, false, INPLACE>), dim3(grid), dim3(256), 0, st, A);
  }
  return hipGetLastError();
}

template <int HMAX>
static hipError_t eval_f64_h(const EvalArgs& A, bool inplace, unsigned grid, hipStream_t st) {
  if constexpr (HMAX >= 128) {
    if (inplace)
      return A.sys.W == 1 ? eval_f64_nw<HMAX, 1, true>(A, grid, st) : eval_f64_nw<HMAX, 2, true>(A, grid, st);
  }
  return A.sys.W == 1 ? eval_f64_nw<HMAX, 1, false>(A, grid, st) : eval_f64_nw<HMAX, 2, false>(A, grid, st);
}

template <int HMAX>
static hipError_t eval_multi_f64_h(const EvalArgs* args, const int64_t* first, int n_sys, unsigned grid,
                                   hipStream_t st) {
  hipLaunchKernelGGL(k_eval_multi_f64<HMAX>, dim3(grid), dim3(256), 0, st, args, first, n_sys);
  return hipGetLastError();
}

hipError_t launch_eval_multi_f64(const EvalArgs* args, const int64_t* first, int n_sys, int hmax,
                                 unsigned grid, hipStream_t st) {
  switch (hmax) {
    case 32: return eval_multi_f64_h<32>(args, first, n_sys, grid, st);
    case 64: return eval_multi_f64_h<64>(args, first, n_sys, grid, st);
    case 128: return eval_multi_f64_h<128>(args, first, n_sys, grid, st);
    case 256: return eval_multi_f64_h<256>(args, first, n_sys, grid, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_eval_f64(const EvalArgs& A, int hmax, bool inplace, unsigned grid, hipStream_t st) {
  if (A.n_items <= 0) return hipSuccess;
  switch (hmax) {
    case 32: return eval_f64_h<32>(A, false, grid, st);
    case 64: return eval_f64_h<64>(A, false, grid, st);
    case 128: return eval_f64_h<128>(A, inplace, grid, st);
    case 256: return eval_f64_h<256>(A, inplace, grid, st);
  }
  return hipErrorInvalidValue;
}

template <int HMAX>
static hipError_t bas_probs_h(const SysDev& S, const MadeDev& M, const uint64_t* pre, const int64_t* Ud, int64_t cap,
                              int k, double* probs, hipStream_t st) {
  const int64_t waves = (cap + 15) / 16;
  const unsigned blocks = (unsigned)((waves + 3) / 4);
  // orbital k's logits see the last hidden layer's units of degree <= k, and a hidden unit
  // of degree d only units of degree <= d below it: in every hidden layer the units of
  // degree <= k, the first ones of the degree-sorted packing
  HiddenCaps caps{};
  for (int l = 0; l < M.L; ++l) {
    const int w = M.nout[l], q = S.n - 1;
    int cnt = 0;
    for (int r = 0; r < q && r < k; ++r) cnt += (w > r) ? (w - r - 1) / q + 1 : 0;   // degree r + 1 <= k
    caps.nob[l] = (cnt + 15) / 16;
  }
  if (S.W == 1)
    hipLaunchKernelGGL((k_bas_probs<HMAX, 1>), dim3(blocks), dim3(256), 0, st, S, M, caps, pre, Ud, cap, k, probs);
  else
    hipLaunchKernelGGL((k_bas_probs<HMAX, 2>), dim3(blocks), dim3(256), 0, st, S, M, caps, pre, Ud, cap, k, probs);
  return hipGetLastError();
}

hipError_t launch_bas_probs(const SysDev& S, const MadeDev& M, int hmax, const uint64_t* pre, const int64_t* Ud,
                            int64_t cap, int k, double* probs, hipStream_t st) {
  switch (hmax) {
    case 32: return bas_probs_h<32>(S, M, pre, Ud, cap, k, probs, st);
    case 64: return bas_probs_h<64>(S, M, pre, Ud, cap, k, probs, st);
    case 128: return bas_probs_h<128>(S, M, pre, Ud, cap, k, probs, st);
    case 256: return bas_probs_h<256>(S, M, pre, Ud, cap, k, probs, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace elocal
