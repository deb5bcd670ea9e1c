// Autoregressive ansatz with bfloat16 parameters on the 16-bit matrix cores
// (v_mfma_f32_16x16x32_f16) and the fused local-energy kernel built on it.
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
// Sparsity: hidden units are packed in ascending degree. A unit of degree m only sees
// units of degree <= m of the layer below (or the bits of orbitals < m, or, for the
// logits of orbital p, hidden units of degree <= p), i.e. a prefix in this order, so
// o-block ob of layer l multiplies only its first kend[l][ob] k-blocks.
//
// Precision: the caller's weights are bfloat16; the packing stores them as fp16, which
// holds every bfloat16 value in [2^-17, 65504] exactly (8 significant bits in fp16's 11),
// so both operand types of the products are fp16 and run at the bfloat16 rate. Layer-0
// inputs are exact 0/1; every later activation a (FP32 after bias and ReLU) is fed as
// hi = fp16(a) plus lo = fp16(a - hi) (a third term in the three-term mode), one MFMA
// per term and weight fragment: two terms represent a to within 2^-22 |a| (fp16 keeps 11
// significant bits; 2^-25 absolute for the smallest values), where two bfloat16 terms
// would leave 2^-16 |a|. Accumulation is FP32; the ratio exp(dA + i dphi), the matrix
// element and every sum are FP64.
#include <algorithm>
#include <type_traits>

#include "elocal_internal.hpp"
#include "kernels.hpp"

namespace elocal {

// Output layer of the BF16 packing: rows 4p..4p+3 hold the logits of orbital p < n - 1 and
// row 4(n - 1) the phase head. The last orbital needs no logits: with no orbital left after
// it exactly one occupation keeps both electron counts reachable, so its conditional is 1.
__device__ __forceinline__ int phase_row_bf16(int n) { return 4 * (n - 1); }

__device__ __forceinline__ bool made_allowed(int n, int L, int l, int o, int k) {
  const int nm1 = n - 1;
  if (l == 0) return (o % nm1) + 1 >= k / 2 + 1;
  if (l < L) return (o % nm1) + 1 >= (k % nm1) + 1;
  if (o == phase_row_bf16(n)) return true;   // phase head sees the whole last layer
  return (o / 4) + 1 > (k % nm1) + 1;
}

// k index (position within the layer's packed input order) of k-slot j of lane group g.
__device__ __forceinline__ int kslot_bf16(int l, int kb, int g, int j) {
  if (l == 0) return 32 * kb + 8 * g + j;
  return 32 * kb + (j < 4 ? 4 * g + j : 16 + 4 * g + (j - 4));
}

// The fp16 pattern of a bf16 value (RNE). Exact for 2^-17 <= |w| <= 65504 (8 significant
// bits fit fp16's 11, and fp16 subnormals reach down to multiples of 2^-24); smaller values
// move by at most 2^-25, larger ones overflow to infinity.
__device__ __forceinline__ unsigned short f16_bits_of_bf16(unsigned short b) {
  const _Float16 h = (_Float16)__uint_as_float((uint32_t)b << 16);
  unsigned short r;
  __builtin_memcpy(&r, &h, 2);
  return r;
}

// Packs the caller's parameters (bf16 bit patterns, natural order) into fp16 MFMA A-operand
// fragments (only the k-blocks each o-block uses) with hidden units in degree order, masked
// entries zeroed; biases to FP32.
__global__ void k_pack_bf16(MadeDev M, ThetaLayout T, const uint16_t* __restrict__ theta,
                            h16x8* __restrict__ frag, float* __restrict__ bias) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = M.n, L = M.L;
  if (gid < M.nfrag * 64u) {
    const int32_t f = (int32_t)(gid >> 6);
    const int lane = gid & 63;
    int l = 0;
    while (l < L && f >= M.foff[l + 1][0]) ++l;
    int ob = 0;
    while (ob + 1 < M.nob[l] && f >= M.foff[l][ob + 1]) ++ob;
    const int kb = f - M.foff[l][ob];
    const int orow = 16 * ob + (lane & 15), g = lane >> 4;
    // original output unit of this row
    const int o = (l < L) ? (orow < M.nout[l] ? sorted_unit(n, M.nout[l], orow) : -1)
                          : (orow < M.nout[l] ? orow : -1);
    unsigned short v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kpos = kslot_bf16(l, kb, g, j);
      int k = -1;
      if (kpos < M.nin[l]) k = (l == 0) ? kpos : sorted_unit(n, M.nin[l], kpos);
      unsigned short bits = 0;
      if (o >= 0 && k >= 0 && made_allowed(n, L, l, o, k)) {
        if (l == L && o == phase_row_bf16(n)) bits = theta[T.offwphi + k];
        else bits = theta[T.offW[l] + (uint32_t)o * M.nin[l] + k];
      }
      v[j] = f16_bits_of_bf16(bits);
    }
    h16x8 out;
    __builtin_memcpy(&out, v, sizeof(out));
    frag[gid] = out;
  }
  if (gid < M.nbias) {
    int l = 0;
    while (l < L && gid >= M.boff[l + 1]) ++l;
    const int orow = gid - M.boff[l];
    unsigned short bits = 0;
    if (orow < M.nout[l]) {
      if (l < L) bits = theta[T.offb[l] + sorted_unit(n, M.nout[l], orow)];
      else bits = (orow == phase_row_bf16(n)) ? theta[T.offbphi] : theta[T.offb[l] + orow];
    }
    bias[gid] = __uint_as_float((uint32_t)bits << 16);
  }
}

__device__ __forceinline__ h16x8 bits_to_h16x8(uint32_t v) {
  uint32_t w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    w[q] = (((v >> (2 * q)) & 1u) * 0x3C00u) | ((((v >> (2 * q + 1)) & 1u) * 0x3C00u) << 16);
  h16x8 r;
  __builtin_memcpy(&r, w, sizeof(r));
  return r;
}

typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));

// ReLU of a pair, then NT fp16 terms whose sum represents each value: t[0] = fp16(a),
// t[1] = fp16(a - t[0]), t[2] = fp16(a - t[0] - t[1]) (one packed convert for the first
// term of both values; each later term is one fused multiply-add with an fp16 operand
// that rounds straight to fp16, a - t[0] being exact in FP32). Two terms leave at most
// 2^-22 |a| for |a| >= 2^-3 and 2^-25 in absolute terms below (fp16 subnormals), three
// terms far less. Values must stay below 65504 (the fp16 range).
template <int NT>
__device__ __forceinline__ void split_pair(float u, float v, uint32_t (&t)[NT]) {
  u = __int_as_float(max(__float_as_int(u), 0));     // ReLU: negative floats are negative ints
  v = __int_as_float(max(__float_as_int(v), 0));
  // a 1.0 the optimiser cannot fold: fma(-t, one, a) then stays one mixed-precision FMA
  float one;
  asm("s_mov_b32 %0, 1.0" : "=s"(one));
  h16x2 h;
  h[0] = (_Float16)u;
  h[1] = (_Float16)v;
  uint32_t hb;
  __builtin_memcpy(&hb, &h, 4);
  // opaque to the optimiser: the residuals below read the packed value, not a second convert
  asm volatile("" : "+v"(hb));
  t[0] = hb;
  if (NT > 1) {
    h16x2 hh;
    __builtin_memcpy(&hh, &hb, 4);
    const float ru = __builtin_fmaf(-(float)hh[0], one, u);
    const float rv = __builtin_fmaf(-(float)hh[1], one, v);
    h16x2 l;
    l[0] = (_Float16)ru;
    l[1] = (_Float16)rv;
    uint32_t lb;
    __builtin_memcpy(&lb, &l, 4);
    t[1] = lb;
    if (NT > 2) {
      asm volatile("" : "+v"(lb));
      h16x2 ll;
      __builtin_memcpy(&ll, &lb, 4);
      const float su = __builtin_fmaf(-(float)ll[0], one, ru);
      const float sv = __builtin_fmaf(-(float)ll[1], one, rv);
      h16x2 m;
      m[0] = (_Float16)su;
      m[1] = (_Float16)sv;
      __builtin_memcpy(&t[NT > 2 ? 2 : 0], &m, 4);
    }
  }
}

// Units 4g..4g+3 of block a and of block a+1 -> the 8 k-slots of the next layer, as NT
// fp16 terms.
template <int NT>
__device__ __forceinline__ void split_relu(const f32x4& a, const f32x4& b, h16x8 (&out)[NT]) {
  uint32_t t[4][NT];
  split_pair<NT>(a[0], a[1], t[0]);
  split_pair<NT>(a[2], a[3], t[1]);
  split_pair<NT>(b[0], b[1], t[2]);
  split_pair<NT>(b[2], b[3], t[3]);
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const uint32_t w[4] = {t[0][i], t[1][i], t[2][i], t[3][i]};
    __builtin_memcpy(&out[i], w, 16);
  }
}

__device__ __forceinline__ int sgpr(int v) { return __builtin_amdgcn_readfirstlane(v); }

// k-range of o-block ob (wave-uniform) from the three packed words of its layer.
__device__ __forceinline__ int kend_packed(uint32_t k0, uint32_t k1, uint32_t k2, int ob) {
  const uint32_t w = ob < 8 ? k0 : ob < 16 ? k1 : k2;
  return (int)((w >> (4 * (ob & 7))) & 15u);
}

__device__ __forceinline__ f32x4 mfma_f16(const h16x8& a, const h16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 load_bias4(const float* bias, uint32_t off) {
  f32x4 r;
  r[0] = bias[off]; r[1] = bias[off + 1]; r[2] = bias[off + 2]; r[3] = bias[off + 3];
  return r;
}

// Every block sees at least its first k-block (kend >= 1, checked when the ansatz is
// packed), so k-block 0 is issued unconditionally in the layers below.
//
// Packing: only the k-blocks an o-block uses are stored, o-block after o-block, so
// fragment kb of o-block ob of layer l is M.foff[l][ob] + kb (kb < kend[l][ob]).
// Where a layer's fragments are read from: LDS when the layer is staged there (lds[l] >= 0
// is then the fragment offset of its first fragment in LDS), else global memory. Each
// layer's code is generated for both sources, so LDS reads are LDS instructions.
template <class Body>
__device__ __forceinline__ void with_layer(const MadeDev& M, const int32_t* lds, const unsigned char* smem, int l,
                                           Body&& body) {
  const int32_t lf = lds ? sgpr(lds[l]) : -1;
  if (lf >= 0) {
    body((const h16x8*)smem + (size_t)lf * 64 - (size_t)M.foff[l][0] * 64, std::true_type{});
  } else {
    body((const h16x8*)M.wfrag, std::false_type{});
  }
}

// Partial staging (the whole network does not fit in LDS) for the widest networks: their
// global-memory layers issue weight loads ahead of the products.
template <int HMAX>
constexpr bool lds_partial_bf16() { return HMAX >= kLdsPartialWidth; }

// Output block ob of the last layer for the NC 16-row tiles (tile c: row r of lane r).
// W: base such that fragment f of the packing is W[f * 64 + lane].
// ke: the block's k-range, fo: its first fragment, bb: the layer's bias offset.
template <int KB, int NT, int NC>
__device__ __forceinline__ void out_block(const h16x8* __restrict__ W, const float* __restrict__ bias, int bb,
                                          const h16x8 (&act)[NT][NC][KB], int ob, int ke, int fo, int lane,
                                          f32x4 (&a)[NC]) {
  const f32x4 b4 = load_bias4(bias, bb + 16 * ob + 4 * (lane >> 4));
#pragma unroll
  for (int c = 0; c < NC; ++c) a[c] = b4;
  const h16x8* wp = W + (size_t)fo * 64 + lane;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    if (kb > 0 && kb >= ke) break;   // the k-range is a prefix: one exit, no test per later k-block
    const h16x8 w = wp[kb * 64];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int i = 0; i < NT; ++i) a[c] = mfma_f16(w, act[i][c][kb], a[c]);
  }
}

// Products of o-block pair (2 kbo, 2 kbo + 1) of hidden layer l >= 1 over the k-blocks its
// mask keeps, into a0 (block 2 kbo) and a1 (block 2 kbo + 1), which arrive holding the
// biases. With PREFETCH (NT = 2) the fragment loads are issued in chunks of four k-blocks,
// one chunk ahead of the products.
// kmin <= kend <= kcap for both blocks of the pair, bounds known where the call is unrolled
// (kbo + 1 and kbo + 2 for the in-place layers, whose host check guarantees them; 1 and KB
// otherwise), so that the k-blocks below kmin run without a test and those from kcap on are
// dropped at compile time.
// ke0, ke1: the blocks' k-ranges; f0, f1: their first fragments.
struct NoWork {
  __device__ __forceinline__ void operator()() const {}
};

template <int KB, int NT, int NC, bool PREFETCH, class Mid = NoWork>
__device__ __forceinline__ void hidden_pair(const h16x8* __restrict__ W, int kbo, int ke0, int ke1, int f0, int f1,
                                            const h16x8 (&act)[NT][NC][KB], int lane, f32x4 (&a0)[NC],
                                            f32x4 (&a1)[NC], int kmin = 1, int kcap = KB, Mid&& mid = Mid{}) {
  ke0 = min(ke0, kcap);
  ke1 = min(ke1, kcap);
  const h16x8* w0p = W + (size_t)f0 * 64 + lane;
  const h16x8* w1p = W + (size_t)f1 * 64 + lane;
  if constexpr (PREFETCH) {
    constexpr int CH = 4, NCH = (KB + CH - 1) / CH;
    h16x8 w0b[NCH][CH], w1b[NCH][CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {   // prologue: chunk 0
      const int kb = j;
      if (kb < kmin || (kb < kcap && kb < ke1)) w1b[0][j] = w1p[kb * 64];
      if (kb < kmin || (kb < kcap && kb < ke0)) w0b[0][j] = w0p[kb * 64];
    }
    mid();   // VALU work of the caller that overlaps the first loads
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      __builtin_amdgcn_sched_barrier(0);
      if (c * CH < kmin || (c * CH < kcap && c * CH < ke1)) {
        if (c + 1 < NCH) {
#pragma unroll
          for (int j = 0; j < CH; ++j) {
            const int kb = (c + 1) * CH + j;
            if (kb < kmin || (kb < kcap && kb < ke1)) w1b[c + 1][j] = w1p[kb * 64];
            if (kb < kmin || (kb < kcap && kb < ke0)) w0b[c + 1][j] = w0p[kb * 64];
          }
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const int kb = c * CH + j;
          if (kb < KB && (kb < kmin || (kb < kcap && kb < ke1))) {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc)
#pragma unroll
              for (int i = 0; i < NT; ++i) a1[cc] = mfma_f16(w1b[c][j], act[i][cc][kb], a1[cc]);
            if (kb < kmin || (kb < kcap && kb < ke0)) {
#pragma unroll
              for (int cc = 0; cc < NC; ++cc)
#pragma unroll
                for (int i = 0; i < NT; ++i) a0[cc] = mfma_f16(w0b[c][j], act[i][cc][kb], a0[cc]);
            }
          }
        }
      }
    }
  } else {
    mid();
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      // ke0 <= ke1 (degrees grow along the layer): one exit once block 1's range ends
      if (kb >= kmin && (kb >= kcap || kb >= ke1)) break;
      const h16x8 w1 = w1p[kb * 64];
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < NT; ++i) a1[c] = mfma_f16(w1, act[i][c][kb], a1[c]);
      if (kb < kmin || (kb < kcap && kb < ke0)) {
        const h16x8 w0 = w0p[kb * 64];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int i = 0; i < NT; ++i) a0[c] = mfma_f16(w0, act[i][c][kb], a0[c]);
      }
    }
  }
}

// In-place hidden layer (see hidden_layer): pairs of output blocks from the highest down.
// FULL: the layer has all KB pairs (nob == 2 KB).
template <int KB, int NT, int NC, bool PREFETCH, bool FULL>
__device__ __forceinline__ void hidden_inplace(const h16x8* __restrict__ W, const float* __restrict__ bias,
                                               uint32_t kp0, uint32_t kp1, uint32_t kp2, int bb, int fo, int nob,
                                               int g, int lane, h16x8 (&act)[NT][NC][KB]) {
  // r0/r1: the products of the pair above, split (ReLU, fp16 terms) while the next pair's
  // first weight loads are in flight; pend: that split, stored once the next pair is done
  h16x8 pend[NT][NC];
  f32x4 r0[NC], r1[NC];
#pragma unroll
  for (int kbo = KB - 1; kbo >= 0; --kbo) {
    if (FULL || 2 * kbo < nob) {
      const int ke0 = kend_packed(kp0, kp1, kp2, 2 * kbo), ke1 = kend_packed(kp0, kp1, kp2, 2 * kbo + 1);
      const int f1 = fo - ke1, f0 = f1 - ke0;
      fo = f0;
      f32x4 a0[NC], a1[NC];
      {
        const f32x4 b0 = load_bias4(bias, bb + 32 * kbo + 4 * g);
        const f32x4 b1 = load_bias4(bias, bb + 32 * kbo + 16 + 4 * g);
#pragma unroll
        for (int c = 0; c < NC; ++c) { a0[c] = b0; a1[c] = b1; }
      }
      const bool above = kbo + 1 < KB && (FULL || 2 * (kbo + 1) < nob);   // pair kbo + 1 exists
      hidden_pair<KB, NT, NC, PREFETCH>(W, kbo, ke0, ke1, f0, f1, act, lane, a0, a1, kbo + 1, kbo + 2, [&] {
        if (above) {
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            h16x8 t[NT];
            split_relu<NT>(r0[c], r1[c], t);
#pragma unroll
            for (int i = 0; i < NT; ++i) pend[i][c] = t[i];
          }
        }
      });
      if (above) {
#pragma unroll
        for (int i = 0; i < NT; ++i)
#pragma unroll
          for (int c = 0; c < NC; ++c) act[i][c][kbo + 1 < KB ? kbo + 1 : 0] = pend[i][c];
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) { r0[c] = a0[c]; r1[c] = a1[c]; }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {   // pair 0 (every layer has it)
    h16x8 t[NT];
    split_relu<NT>(r0[c], r1[c], t);
#pragma unroll
    for (int i = 0; i < NT; ++i) act[i][c][0] = t[i];
  }
}

// Hidden layer l >= 1. Without INPLACE the outputs go to a second activation array. With
// INPLACE they overwrite the inputs: pairs run from the last to the first, and the
// result of pair j is held back until pair j - 1 is done, then stored in k-slot j. This
// is exact when no pair j reads beyond k-block j + 1 (kend of its second block <= j + 2,
// which the host checks for every hidden layer): pair j then never sees a slot that was
// already overwritten, and slot j + 1 is free once pair j is done.
template <int HMAX, int NT, int NC, bool INPLACE, bool PREFETCH>
__device__ __forceinline__ void hidden_layer(const MadeDev& M, const h16x8* __restrict__ W,
                                             const float* __restrict__ bias, int l, int lane,
                                             h16x8 (&act)[NT][NC][HMAX / 32]) {
  constexpr int KB = HMAX / 32;
  const int g = lane >> 4, nob = sgpr(M.nob[l]);
  // the layer's k-ranges from three packed words, its bias offset, and fragment offsets as
  // a running sum (a hidden layer's width is a multiple of 32: its blocks come in pairs)
  const uint32_t kp0 = (uint32_t)sgpr((int)M.kpack[l][0]), kp1 = (uint32_t)sgpr((int)M.kpack[l][1]),
                 kp2 = (uint32_t)sgpr((int)M.kpack[l][2]);
  const int bb = sgpr((int)M.boff[l]);
  if constexpr (INPLACE) {
    // a layer of the full width has every pair: no test per pair (a runtime test there costs
    // register moves at every join)
    if (nob == 2 * KB)
      hidden_inplace<KB, NT, NC, PREFETCH, true>(W, bias, kp0, kp1, kp2, bb, sgpr(M.foff[l][nob]), nob, g, lane, act);
    else
      hidden_inplace<KB, NT, NC, PREFETCH, false>(W, bias, kp0, kp1, kp2, bb, sgpr(M.foff[l][nob]), nob, g, lane, act);
  } else {
    // (the narrower networks that run out of place keep four waves per SIMD, which hide
    // the table reads; there, direct reads measured faster than the packed words)
    h16x8 nxt[NT][NC][KB];
#pragma unroll
    for (int kbo = 0; kbo < KB; ++kbo) {
      if (2 * kbo < nob) {
        const int ke0 = sgpr(M.kend[l][2 * kbo]), ke1 = sgpr(M.kend[l][2 * kbo + 1]);
        const int f0 = sgpr(M.foff[l][2 * kbo]), f1 = sgpr(M.foff[l][2 * kbo + 1]);
        f32x4 a0[NC], a1[NC];
        {
          const f32x4 b0 = load_bias4(bias, bb + 32 * kbo + 4 * g);
          const f32x4 b1 = load_bias4(bias, bb + 32 * kbo + 16 + 4 * g);
#pragma unroll
          for (int c = 0; c < NC; ++c) { a0[c] = b0; a1[c] = b1; }
        }
        hidden_pair<KB, NT, NC, PREFETCH>(W, kbo, ke0, ke1, f0, f1, act, lane, a0, a1);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          h16x8 t[NT];
          split_relu<NT>(a0[c], a1[c], t);
#pragma unroll
          for (int i = 0; i < NT; ++i) nxt[i][c][kbo] = t[i];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) act[i][c][kb] = nxt[i][c][kb];
  }
}

// Runs the network on NC 16-row tiles (tile c: row r of lane r) and calls epi(ob, a[NC])
// for the output blocks ob >= ob_first (earlier blocks belong to orbitals the caller does
// not need). Hidden activations are carried as NT fp16 terms (one MFMA per term and
// weight fragment). lds: per-layer LDS placement (see with_layer; nullptr: every layer in
// global memory). With XLUT the layer-0 operands come from the LDS table xlut (16 entries
// of 4 input bits), else they are expanded from the bits in registers.
template <int HMAX, int NW, int NT, int NC, bool XLUT = false, bool INPLACE = false, class Epi>
__device__ __forceinline__ void mlp_bf16(const MadeDev& M, const int32_t* lds, const unsigned char* smem,
                                         const float* __restrict__ bias, const uint64_t (&xr)[NC][NW], int lane,
                                         int ob_first, const uint64_t* xlut, Epi&& epi) {
  constexpr int KB = HMAX / 32;
  constexpr bool PF = lds_partial_bf16<HMAX>() && NT == 2;
  const int g = lane >> 4;
  h16x8 act[NT][NC][KB];
  // ---- layer 0: exact 0/1 inputs, one MFMA per fragment
  {
    const int nk = M.nk[0], nob = M.nob[0];
    h16x8 xin[NC][4];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const uint32_t b8 = kb < nk ? bits8_at<NW>(xr[c], 32 * kb + 8 * g) : 0u;
        if (XLUT) {
          const uint64_t w2[2] = {xlut[b8 & 15u], xlut[b8 >> 4]};
          __builtin_memcpy(&xin[c][kb], w2, 16);
        } else {
          xin[c][kb] = bits_to_h16x8(b8);
        }
      }
    with_layer(M, lds, smem, 0, [&](const h16x8* W, auto in_lds) {
      // global memory with PF: the fragments of pair kbo + 1 are loaded while pair kbo is
      // multiplied (two buffers, all of a pair's at most 4 k-blocks at once)
      constexpr bool G0 = !decltype(in_lds)::value && PF;
      h16x8 wb[G0 ? 2 : 1][2][4];
      // the two blocks of a pair share one k-range (the host pads the pair's first block)
      auto load_pair = [&](int kbo, h16x8 (&dst)[2][4]) {
        const int ke = sgpr(M.kend[0][2 * kbo + 1]);
        const h16x8* w0p = W + (size_t)sgpr(M.foff[0][2 * kbo]) * 64 + lane;
        const h16x8* w1p = W + (size_t)sgpr(M.foff[0][2 * kbo + 1]) * 64 + lane;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          if (kb > 0 && kb >= ke) break;
          dst[1][kb] = w1p[kb * 64];
          dst[0][kb] = w0p[kb * 64];
        }
      };
      if constexpr (G0) load_pair(0, wb[0]);
#pragma unroll
      for (int kbo = 0; kbo < KB; ++kbo) {
        if (2 * kbo < nob) {
          const int ke = sgpr(M.kend[0][2 * kbo + 1]);   // both blocks of the pair
          f32x4 a0[NC], a1[NC];
          {
            const f32x4 b0 = load_bias4(bias, M.boff[0] + 32 * kbo + 4 * g);
            const f32x4 b1 = load_bias4(bias, M.boff[0] + 32 * kbo + 16 + 4 * g);
#pragma unroll
            for (int c = 0; c < NC; ++c) { a0[c] = b0; a1[c] = b1; }
          }
          if constexpr (G0) {
            if (kbo + 1 < KB && 2 * (kbo + 1) < nob) load_pair(kbo + 1 < KB ? kbo + 1 : 0, wb[(kbo + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
              if (kb > 0 && kb >= ke) break;
#pragma unroll
              for (int c = 0; c < NC; ++c) a1[c] = mfma_f16(wb[kbo & 1][1][kb], xin[c][kb], a1[c]);
#pragma unroll
              for (int c = 0; c < NC; ++c) a0[c] = mfma_f16(wb[kbo & 1][0][kb], xin[c][kb], a0[c]);
            }
          } else {
            const h16x8* w0p = W + (size_t)sgpr(M.foff[0][2 * kbo]) * 64 + lane;
            const h16x8* w1p = W + (size_t)sgpr(M.foff[0][2 * kbo + 1]) * 64 + lane;
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
              if (kb > 0 && kb >= ke) break;
              const h16x8 w1 = w1p[kb * 64];
#pragma unroll
              for (int c = 0; c < NC; ++c) a1[c] = mfma_f16(w1, xin[c][kb], a1[c]);
              const h16x8 w0 = w0p[kb * 64];
#pragma unroll
              for (int c = 0; c < NC; ++c) a0[c] = mfma_f16(w0, xin[c][kb], a0[c]);
            }
          }
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            h16x8 t[NT];
            split_relu<NT>(a0[c], a1[c], t);
#pragma unroll
            for (int i = 0; i < NT; ++i) act[i][c][kbo] = t[i];
          }
        }
      }
    });
  }
  // ---- hidden layers 1..L-1
  for (int l = 1; l < M.L; ++l) {
    // the widest networks issue a chunk of fragment loads ahead of the products from LDS
    // as from global memory (one wait per chunk instead of one per fragment)
    with_layer(M, lds, smem, l, [&](const h16x8* W, auto) {
      hidden_layer<HMAX, NT, NC, INPLACE, PF>(M, W, bias, l, lane, act);
    });
  }
  // ---- output layer, block by block into the epilogue
  with_layer(M, lds, smem, M.L, [&](const h16x8* W, auto) {
    const int nob = M.nob[M.L];
    if constexpr (PF) {
      // the fragments of block ob + 1 are loaded while block ob is multiplied and its
      // epilogue runs (two buffers, all of a block's k-blocks at once)
      const int l = M.L;
      h16x8 wv[2][KB];
      // k-ranges from three packed words read once, fragment offsets as a running sum
      const uint32_t kp0 = (uint32_t)sgpr((int)M.kpack[l][0]), kp1 = (uint32_t)sgpr((int)M.kpack[l][1]),
                     kp2 = (uint32_t)sgpr((int)M.kpack[l][2]);
      const int bbase = sgpr((int)M.boff[l]);
      auto load_block = [&](int ke, int fo, h16x8 (&dst)[KB]) {
        const h16x8* wp = W + (size_t)fo * 64 + lane;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          if (kb > 0 && kb >= ke) break;
          dst[kb] = wp[kb * 64];
        }
      };
      auto run_block = [&](int ob, int ke, const h16x8 (&wsrc)[KB]) {
        f32x4 a[NC];
        const f32x4 b4 = load_bias4(bias, bbase + 16 * ob + 4 * g);
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c] = b4;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          if (kb > 0 && kb >= ke) break;
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int i = 0; i < NT; ++i) a[c] = mfma_f16(wsrc[kb], act[i][c][kb], a[c]);
        }
        epi(ob, a);
      };
      int ob = sgpr(ob_first);
      int fo = ob < nob ? sgpr(M.foff[l][ob]) : 0;   // first fragment of block ob
      int ke = kend_packed(kp0, kp1, kp2, ob);
      if (ob < nob) load_block(ke, fo, wv[0]);
#pragma unroll 1
      while (ob < nob) {
        int fo1 = fo + ke, ke1 = kend_packed(kp0, kp1, kp2, ob + 1);
        if (ob + 1 < nob) load_block(ke1, fo1, wv[1]);
        __builtin_amdgcn_sched_barrier(0);
        run_block(ob, ke, wv[0]);
        if (++ob >= nob) break;
        fo = fo1;
        ke = ke1;
        fo1 = fo + ke;
        ke1 = kend_packed(kp0, kp1, kp2, ob + 1);
        if (ob + 1 < nob) load_block(ke1, fo1, wv[0]);
        __builtin_amdgcn_sched_barrier(0);
        run_block(ob, ke, wv[1]);
        ++ob;
        fo = fo1;
        ke = ke1;
      }
    } else {
      // (four waves per SIMD: direct table reads, as in the out-of-place hidden layers)
      const int l = M.L;
#pragma unroll 1
      for (int ob = sgpr(ob_first); ob < nob; ++ob) {
        f32x4 acc[NC];
        out_block<KB, NT, NC>(W, bias, M.boff[l], act, ob, sgpr(M.kend[l][ob]), sgpr(M.foff[l][ob]), lane, acc);
        epi(ob, acc);
      }
    }
  });
}

// Per-row state of the epilogue at the lane's current orbital p: the row's occupation
// bits from orbital p on (bit 0 = alpha of p) and the electrons of each spin before p.
// Advanced by four orbitals per output block.
template <int NW>
struct RowCursor {
  uint64_t bits[NW];
  int cu, cd;
};

template <int NW>
__device__ __forceinline__ RowCursor<NW> cursor_at(const uint64_t (&x)[NW], int p) {
  RowCursor<NW> r;
  r.cu = count_spin_below<NW>(x, p, 0);
  r.cd = count_spin_below<NW>(x, p, 1);
  const int k = 2 * p;   // < 64 NW for every orbital the epilogue visits
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    uint64_t v = 0;
#pragma unroll
    for (int u = w; u < NW; ++u) {
      const int sh = 64 * (u - w) - k;   // bit i of word u lands at 64(u - w) + i - k
      if (sh >= 0 && sh < 64) v |= x[u] << sh;
      else if (sh < 0 && sh > -64) v |= x[u] >> (-sh);
    }
    r.bits[w] = v;
  }
  return r;
}

template <int NW>
__device__ __forceinline__ void cursor_advance4(RowCursor<NW>& r, uint32_t b8) {
  r.cu += __popc(b8 & 0x55u);
  r.cd += __popc(b8 & 0xAAu);
#pragma unroll
  for (int w = 0; w < NW; ++w) r.bits[w] = (r.bits[w] >> 8) | (w + 1 < NW ? r.bits[w + 1] << 56 : 0ull);
}

constexpr float kLog2e = 1.4426950408889634f;
constexpr double kLn2 = 0.6931471805599453094;

// log2 p_p(s_p) of the row at the cursor's orbital, then advance the cursor by four
// orbitals. The softmax runs over the occupations that keep both electron counts
// reachable: alpha must be taken if cu < ta (= n_alpha - orbitals after p), may be
// taken if cu < na (same for beta). Base 2 on the native exp2/log2 units (one rescale
// to natural log per row, by the caller), shifted by the taken occupation's logit:
// log2 p = -log2(sum over allowed s of 2^(y_s - y_taken)), where the taken term is 1, so
// the sum is >= 1; it overflows only when p is below 2^-128, and then gives -inf, the
// right limit for a ratio (that entry's amplitude is 0 to double precision).
template <int NW>
__device__ __forceinline__ float cond_log2p_step(RowCursor<NW>& rc, int ta, int tb, int na, int nb,
                                                 const f32x4& z) {
  const uint32_t b8 = (uint32_t)rc.bits[0] & 0xFFu;
  const bool a_must = rc.cu < ta, a_may = rc.cu < na;
  const bool b_must = rc.cd < tb, b_may = rc.cd < nb;
  const bool ok0 = !a_must && !b_must, ok1 = a_may && !b_must;
  const bool ok2 = !a_must && b_may, ok3 = a_may && b_may;
  // the taken logit in log2 units; each exponent is one fused multiply-add
  const float z01 = (b8 & 1u) ? z[1] : z[0];
  const float z23 = (b8 & 1u) ? z[3] : z[2];
  const float ys = ((b8 & 2u) ? z23 : z01) * kLog2e;
  const float e0 = ok0 ? __builtin_amdgcn_exp2f(__builtin_fmaf(z[0], kLog2e, -ys)) : 0.f;
  const float e1 = ok1 ? __builtin_amdgcn_exp2f(__builtin_fmaf(z[1], kLog2e, -ys)) : 0.f;
  const float e2 = ok2 ? __builtin_amdgcn_exp2f(__builtin_fmaf(z[2], kLog2e, -ys)) : 0.f;
  const float e3 = ok3 ? __builtin_amdgcn_exp2f(__builtin_fmaf(z[3], kLog2e, -ys)) : 0.f;
  const float sum = (e0 + e1) + (e2 + e3);
  cursor_advance4<NW>(rc, b8);
  return -__builtin_amdgcn_logf(sum);
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int row_min(int v) {   // least over the lane's 16-lane row
#pragma unroll
  for (int off = 8; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off));
  return v;
}

// ----------------------------------------------------------------------------- sample pass
// A(x), phi(x) and the per-orbital log p_p(s_p) of every sample (32 samples per wave step).
template <int HMAX, int NW, int NT>
__global__ void __launch_bounds__(256) k_rows_bf16(RowsArgs P) {
  const int lane = threadIdx.x & 63, g = lane >> 4, r16 = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t b0 = wave * 32;
  const int64_t Bn = P.count ? min(P.B, *P.count) : P.B;
  if (b0 >= Bn) return;
  const MadeDev& M = P.made;
  const int n = P.sys.n, na = P.sys.na, nb = P.sys.nb;
  const float* bias = (const float*)M.bias;
  uint64_t xr[2][NW];
  int64_t rb[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    rb[c] = b0 + 16 * c + r16;
    const int64_t bb = rb[c] < Bn ? rb[c] : b0;
#pragma unroll
    for (int w = 0; w < NW; ++w) xr[c][w] = P.x[bb * NW + w];
  }
  const int ob_phi = phase_row_bf16(n) >> 4, g_phi = (phase_row_bf16(n) & 15) >> 2;
  double A[2] = {0.0, 0.0};
  float zp[2] = {0.f, 0.f};
  RowCursor<NW> rc[2] = {cursor_at<NW>(xr[0], min(g, n - 1)), cursor_at<NW>(xr[1], min(g, n - 1))};
  mlp_bf16<HMAX, NW, NT, 2>(M, nullptr, nullptr, bias, xr, lane, 0, nullptr, [&](int ob, const f32x4 (&a)[2]) {
    const int p = 4 * ob + g;
    if (p < n - 1) {   // the last orbital's conditional is 1
      const int ta = na - (n - p - 1), tb = nb - (n - p - 1);
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const float lp = cond_log2p_step<NW>(rc[c], ta, tb, na, nb, a[c]);
        A[c] += (double)lp;
        if (rb[c] < Bn) P.lpx[rb[c] * n + p] = lp;     // log2 units
      }
    }
    if (ob == ob_phi && g == g_phi) { zp[0] = a[0][0]; zp[1] = a[1][0]; }
  });
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    A[c] += __shfl_xor(A[c], 16);
    A[c] += __shfl_xor(A[c], 32);
    zp[c] = __shfl(zp[c], g_phi * 16 + r16);
  }
  if (g < 2) {
    const int c = g;
    if (rb[c] < Bn) {
      P.zphi[rb[c]] = (double)zp[c];
      if (P.logpsi) {
        const double sig = 1.0 / (1.0 + exp(-(double)zp[c]));
        P.logpsi[2 * rb[c]] = 0.5 * kLn2 * A[c];
        P.logpsi[2 * rb[c] + 1] = 2.0 * M_PI * sig;
      }
    }
  }
}

// ----------------------------------------------------------------------------- fused eval
struct WaveCtxBF16 {
  SampleCtx c;
};
static_assert(sizeof(WaveCtxBF16) == kWaveCtxBytesBF16, "per-wave LDS context size");

// What a wave keeps of the sample its current work item belongs to.
template <int NW>
struct SampleState {
  int64_t b;
  uint64_t xs[NW];
  double sig_x, ed;
  double sfx;   // lane q: sum_{p >= q} log2 p_p(s_p) of the sample (0 from the last orbital on)
  const double* Fs;
};

// Entry generators of the fused kernel. Entry t of a sample's list (t = 0 is the sample
// itself and is handled outside the kernel) gives x' and H_{x x'}.
//
// Slater--Condon route: the canonical list of single and double excitations.
struct ScGen {
  __device__ __forceinline__ static uint32_t length(const EvalArgs& P) { return P.sys.C; }
  template <int NW>
  __device__ __forceinline__ static double entry(const EvalArgs& P, const SampleCtx& c, const uint64_t (&xs)[NW],
                                                 const double* Fs, double ed, uint32_t t, uint64_t (&xo)[NW]) {
    const Excitation e = unrank(P.sys, c, t);
    const int sg = apply_excitation<NW>(xs, e, xo);
    const double v = excitation_value(P.sys, e, Fs, ed);
    return sg < 0 ? -v : v;
  }
};

// Pauli-string route (Results, Algorithm 1): entry t is unique flip mask t; x' = x XOR
// mask and H_{x x'} = sum over the strings c X^mask Z^z of that mask of c (-1)^|z & x'|.
// A flip that leaves the (n_alpha, n_beta) sector gets H = 0 exactly (there the ansatz is
// zero; its strings' coefficients cancel up to rounding).
struct PauliGen {
  __device__ __forceinline__ static uint32_t length(const EvalArgs& P) { return P.pl_len; }
  template <int NW>
  __device__ __forceinline__ static double entry(const EvalArgs& P, const SampleCtx&, const uint64_t (&xs)[NW],
                                                 const double*, double, uint32_t t, uint64_t (&xo)[NW]) {
    const uint64_t m = P.pl_mask[t];
    xo[0] = xs[0] ^ m;
#pragma unroll
    for (int w = 1; w < NW; ++w) xo[w] = xs[w];
    const uint64_t A = 0x5555555555555555ull;
    if (__popcll(xo[0] & A) != __popcll(xs[0] & A) || __popcll(xo[0] & ~A) != __popcll(xs[0] & ~A)) return 0.0;
    double h = 0.0;
    for (uint32_t k = P.pl_off[t], e = P.pl_off[t + 1]; k < e; ++k) {
      const double c = P.pl_coef[k];
      h += (__popcll(P.pl_z[k] & xo[0]) & 1) ? -c : c;
    }
    return h;
  }
};

// H exp(dA ln2 / 2 + i 2 pi (sigmoid(zp) - sig_x)) in FP64. The phase difference 2 pi d has
// |d| < 1, so sincospi needs no large-argument reduction; the magnitude with dA in log2
// units is exp2(dA / 2). Not inlined (nor is the sample's sigmoid): inlined, the compiler
// keeps the constants of the FP64 functions in registers across the whole kernel, and at
// four waves per SIMD they spill to scratch memory.
__device__ __attribute__((noinline)) double sigmoid64(double z) { return 1.0 / (1.0 + exp(-z)); }

__device__ __attribute__((noinline)) double2 ratio_term(double hv, float zp, double sig_x, double dA) {
  const double d = 1.0 / (1.0 + exp(-(double)zp)) - sig_x;
  double sn, cs;
  sincospi(2.0 * d, &sn, &cs);
  const double mag = hv * exp2(0.5 * dA);
  return make_double2(mag * cs, mag * sn);
}

// One work item = one sample and P.tpi consecutive groups of 64 list entries. Per group:
// every lane generates one entry (x', H_{x'x} in FP64, first changed orbital); the
// network runs in 4 / NC passes of NC 16-row tiles over the 64 entries; every lane then
// forms H exp(dA + i dphi) in FP64 for its own entry. The item's partial sum (fixed
// order) goes to P.partial[item].
template <int HMAX, int NW, int NT, bool INPLACE = false, class Gen = ScGen,
          int NC = eval_cols_default_bf16(HMAX, NT)>
__device__ __forceinline__ void eval_item_bf16(const EvalArgs& P, const int32_t* lds, const unsigned char* smem,
                                               const float* __restrict__ bias, const uint64_t* xlut,
                                               WaveCtxBF16& wc, int64_t item, SampleState<NW>& st, int lane) {
  const MadeDev& M = P.made;
  const SysDev& S = P.sys;
  const int g = lane >> 4, r16 = lane & 15;
  const int n = S.n, na = S.na, nb = S.nb;
  const int ob_phi = phase_row_bf16(n) >> 4, g_phi = (phase_row_bf16(n) & 15) >> 2;
  const int64_t b = item / P.ips;
  const uint32_t seg = (uint32_t)(item % P.ips);
  if (b != st.b) {
    wave_sync_lds();
#pragma unroll
    for (int w = 0; w < NW; ++w) st.xs[w] = P.x[b * NW + w];
    build_ctx<NW>(S, st.xs, wc.c, lane);
    {
      // suffix sums of the sample's log2 p in FP64 (a fixed shuffle tree)
      double v = lane < n - 1 ? (double)P.lpx[b * n + lane] : 0.0;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const double u = __shfl_down(v, off);
        if (lane + off < 64) v += u;
      }
      st.sfx = v;   // lanes >= n - 1 sum nothing: 0
    }
    wave_sync_lds();
    st.sig_x = sigmoid64(P.zphi[b]);
    st.ed = P.ediag[b];
    st.Fs = P.F + (size_t)b * (S.nSa + S.nSb);
    st.b = b;
  }
  const uint64_t(&xs)[NW] = st.xs;
  const uint32_t len = Gen::length(P);
  double acc_re = 0.0, acc_im = 0.0;
  for (uint32_t grp = 0; grp < P.tpi; ++grp) {
    const uint32_t t0 = 1u + (seg * P.tpi + grp) * 64u;
    if (t0 >= len) break;
    // ---- generate this lane's entry
    const uint32_t t = t0 + lane;
    uint64_t xo[NW];
    double hv = 0.0;
    if (t < len) {
      hv = Gen::template entry<NW>(P, wc.c, xs, st.Fs, st.ed, t, xo);
    } else {
#pragma unroll
      for (int w = 0; w < NW; ++w) xo[w] = xs[w];
    }
    const int p0o = first_diff_orbital<NW>(xs, xo, n);
    // the sample's part of this entry's dA, from the lane that holds orbital p0o
    const double sfx_own = __shfl(st.sfx, min(p0o, 63));
    // the first changed orbital, least over each 16-lane row (a tile's rows): output blocks
    // below a tile's least one hold only orbitals that all its rows share with x
    const int p0_row = row_min(p0o);
    double dA_own = 0.0;
    float zp_own = 0.f;
    // ---- network on entries 16 NC h .. 16 NC (h + 1) - 1 (not unrolled: one copy of the
    // network code)
#pragma unroll 1
    for (int h = 0; h < 4 / NC; ++h) {
      uint64_t xr[NC][NW];
      int p0[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int src = 16 * NC * h + 16 * c + r16;
#pragma unroll
        for (int w = 0; w < NW; ++w) xr[c][w] = __shfl(xo[w], src);
        p0[c] = __shfl(p0o, src);
      }
      double dA[NC];
      float zp[NC];
      RowCursor<NW> rc[NC];
      int ob_first = __builtin_amdgcn_readlane(p0_row, 16 * NC * h);
#pragma unroll
      for (int c = 1; c < NC; ++c) ob_first = min(ob_first, __builtin_amdgcn_readlane(p0_row, 16 * NC * h + 16 * c));
      ob_first = sgpr(min(ob_first >> 2, ob_phi));
      const int pfirst = min(4 * ob_first + g, n - 1);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        dA[c] = 0.0;
        zp[c] = 0.f;
        rc[c] = cursor_at<NW>(xr[c], pfirst);
      }
      mlp_bf16<HMAX, NW, NT, NC, true, INPLACE>(M, lds, smem, bias, xr, lane, ob_first, xlut,
                                                 [&](int ob, const f32x4 (&a)[NC]) {
        const int p = 4 * ob + g;
        if (p < n - 1) {   // the last orbital's conditional is 1
          const int ta = na - (n - p - 1), tb = nb - (n - p - 1);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const float lp = cond_log2p_step<NW>(rc[c], ta, tb, na, nb, a[c]);
            float d = p >= p0[c] ? lp : 0.f;
            asm volatile("" : "+v"(d));   // keeps the select in 32 bits (before the convert)
            dA[c] += (double)d;     // sum over p >= p0 of log2 p(x'); x's part is subtracted below
          }
        }
        // the phase row is the output layer's last row (block ob_phi, the last one run): the
        // value the last block leaves in lane group g_phi is the phase logit
#pragma unroll
        for (int c = 0; c < NC; ++c) zp[c] = a[c][0];
      });
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        dA[c] += __shfl_xor(dA[c], 16);
        dA[c] += __shfl_xor(dA[c], 32);
        zp[c] = __shfl(zp[c], g_phi * 16 + r16);
      }
      if (lane / (16 * NC) == h) {
        const int c = (lane >> 4) % NC;
        double dsel = dA[0];
        float zsel = zp[0];
#pragma unroll
        for (int cc = 1; cc < NC; ++cc)
          if (c == cc) { dsel = dA[cc]; zsel = zp[cc]; }
        dA_own = dsel - (p0o < n ? sfx_own : 0.0);
        zp_own = zsel;
      }
    }
    // ---- FP64 ratio and accumulation, one entry per lane (an entry with H = 0 adds
    // nothing; skipping it also keeps an infinite ratio of a zero-amplitude x' out)
    if (t < len && hv != 0.0) {
      const double2 r = ratio_term(hv, zp_own, st.sig_x, dA_own);
      acc_re += r.x;
      acc_im += r.y;
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

// Block shape of the fused kernels: one block per CU, so the whole 160 KiB of LDS can
// hold the packed weights of one ansatz (waves per block: eval_waves_bf16).

// Copies the packed weights of every staged layer (lds[l] >= 0: fragment offset in LDS)
// and the biases into LDS.
__device__ __forceinline__ void stage_weights(const MadeDev& M, const int32_t* lds, unsigned char* smem,
                                              uint32_t bias_off) {
  h16x8* sw = (h16x8*)smem;
  const h16x8* gw = (const h16x8*)M.wfrag;
  for (int l = 0; l <= M.L; ++l) {
    const int32_t lf = lds[l];
    if (lf < 0) continue;
    const uint32_t f0 = (uint32_t)M.foff[l][0], nf = (uint32_t)M.foff[l][M.nob[l]] - f0;
    for (uint32_t i = threadIdx.x; i < nf * 64u; i += blockDim.x) sw[(size_t)lf * 64 + i] = gw[(size_t)f0 * 64 + i];
  }
  float* sb = (float*)(smem + bias_off);
  const float* gb = (const float*)M.bias;
  for (uint32_t i = threadIdx.x; i < M.nbias; i += blockDim.x) sb[i] = gb[i];
}

// Fills the input-expansion table (every thread of the block takes part; the caller
// synchronises the block before the table is read): entry v (4 bits) holds the four fp16
// values bit j of v ? 1 : 0.
__device__ __forceinline__ uint64_t* fill_xlut(unsigned char* smem, uint32_t lut_off) {
  uint64_t* lut = (uint64_t*)(smem + lut_off);
  for (uint32_t v = threadIdx.x; v < 16u; v += blockDim.x) {
    uint64_t e = 0;
    for (int j = 0; j < 4; ++j) e |= (uint64_t)(((v >> j) & 1u) * 0x3C00u) << (16 * j);
    lut[v] = e;
  }
  return lut;
}

// One system; a persistent grid strides over the work items, one wave per item. With
// LDSW the layers the host placed in LDS (P.lds_frag) and the biases are first staged.
template <int HMAX, int NW, int NT, bool LDSW, bool INPLACE, int NC>
__global__ void __launch_bounds__(64 * eval_waves_bf16(HMAX, NT, NC), 1) k_eval_bf16(EvalArgs P) {
  const int kEvalWaves = blockDim.x >> 6;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int lane = threadIdx.x & 63, wid = sgpr(threadIdx.x >> 6);
  const float* bias = (const float*)P.made.bias;
  const uint64_t* xlut = fill_xlut(smem, P.lds_lut_off);
  if (LDSW) {
    stage_weights(P.made, P.lds_frag, smem, P.lds_bias_off);
    bias = (const float*)(smem + P.lds_bias_off);
  }
  __syncthreads();
  WaveCtxBF16& wc = ((WaveCtxBF16*)(smem + P.lds_ctx_off))[wid];
  SampleState<NW> st;
  st.b = -1;
  for (int64_t item = (int64_t)blockIdx.x * kEvalWaves + wid; item < P.n_items;
       item += (int64_t)gridDim.x * kEvalWaves)
    eval_item_bf16<HMAX, NW, NT, INPLACE, ScGen, NC>(P, LDSW ? P.lds_frag : nullptr, smem, bias, xlut, wc, item, st,
                                                    lane);
}

// Pauli-string route: the fused kernel over the unique flip masks of every sample (one
// word per determinant: n <= 32).
template <int HMAX, int NT, bool LDSW>
__global__ void __launch_bounds__(64 * eval_waves_bf16(HMAX, NT, eval_cols_default_bf16(HMAX, NT)), 1)
    k_eval_pauli_bf16(EvalArgs P) {
  const int kEvalWaves = blockDim.x >> 6;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int lane = threadIdx.x & 63, wid = sgpr(threadIdx.x >> 6);
  const float* bias = (const float*)P.made.bias;
  const uint64_t* xlut = fill_xlut(smem, P.lds_lut_off);
  if (LDSW) {
    stage_weights(P.made, P.lds_frag, smem, P.lds_bias_off);
    bias = (const float*)(smem + P.lds_bias_off);
  }
  __syncthreads();
  WaveCtxBF16& wc = ((WaveCtxBF16*)(smem + P.lds_ctx_off))[wid];
  SampleState<1> st;
  st.b = -1;
  for (int64_t item = (int64_t)blockIdx.x * kEvalWaves + wid; item < P.n_items;
       item += (int64_t)gridDim.x * kEvalWaves)
    eval_item_bf16<HMAX, 1, NT, false, PauliGen>(P, LDSW ? P.lds_frag : nullptr, smem, bias, xlut, wc, item, st,
                                                 lane);
}

// Several systems in one persistent launch. Work is cut into chunks of kEvalWaves items
// (one per wave of a block) that never straddle two systems; system s owns chunks
// [first[s], first[s+1]). Blocks stride over the chunks, so every block's share mixes
// the systems in proportion and no system leaves a tail of its own. With LDSW a block
// restages the weights whenever its next chunk belongs to another system (every system's
// staged layers, biases, wave contexts and input table share one LDS layout: the offsets
// of system 0's arguments).
template <int HMAX, int NT, bool LDSW, bool INPLACE, int NC>
__global__ void __launch_bounds__(64 * eval_waves_bf16(HMAX, NT, NC), 1)
    k_eval_multi_bf16(const EvalArgs* __restrict__ args, const int64_t* __restrict__ first, int n_sys) {
  const int kEvalWaves = blockDim.x >> 6;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int lane = threadIdx.x & 63, wid = sgpr(threadIdx.x >> 6);
  const uint32_t bias_off = args[0].lds_bias_off, ctx_off = args[0].lds_ctx_off;
  WaveCtxBF16& wc = ((WaveCtxBF16*)(smem + ctx_off))[wid];
  SampleState<1> st1;
  SampleState<2> st2;
  st1.b = st2.b = -1;
  int cur = -1;
  const float* bias = nullptr;
  const uint64_t* xlut = fill_xlut(smem, args[0].lds_lut_off);
  __syncthreads();
  const int64_t chunks = first[n_sys];
  for (int64_t chunk = blockIdx.x; chunk < chunks; chunk += gridDim.x) {
    int s = 0;
    while (s + 1 < n_sys && chunk >= first[s + 1]) ++s;
    s = sgpr(s);
    const EvalArgs& P = args[s];
    if (s != cur) {
      cur = s;
      st1.b = st2.b = -1;
      if (LDSW) {
        __syncthreads();   // every wave is done with the previous system's weights
        stage_weights(P.made, P.lds_frag, smem, bias_off);
        __syncthreads();
        bias = (const float*)(smem + bias_off);
      } else {
        bias = (const float*)P.made.bias;
      }
    }
    const int64_t local = (chunk - first[s]) * kEvalWaves + wid;
    if (local < P.n_items) {
      const int32_t* lds = LDSW ? P.lds_frag : nullptr;
      if (P.sys.W == 1) eval_item_bf16<HMAX, 1, NT, INPLACE, ScGen, NC>(P, lds, smem, bias, xlut, wc, local, st1, lane);
      else eval_item_bf16<HMAX, 2, NT, INPLACE, ScGen, NC>(P, lds, smem, bias, xlut, wc, local, st2, lane);
    }
  }
}

// ----------------------------------------------------------------------------- launchers
hipError_t launch_pack_bf16(const MadeDev& M, const ThetaLayout& T, const uint16_t* theta,
                            void* frag, float* bias, hipStream_t st) {
  const uint32_t total = M.nfrag * 64u > M.nbias ? M.nfrag * 64u : M.nbias;
  hipLaunchKernelGGL(k_pack_bf16, dim3((total + 255) / 256), dim3(256), 0, st, M, T, theta,
                     (h16x8*)frag, bias);
  return hipGetLastError();
}

// Calls f(integral_constant<HMAX>, integral_constant<NT>) for the runtime width class
// and activation-term count.
template <class F>
static hipError_t dispatch_shape(int hmax, int nt, F&& f) {
  using std::integral_constant;
  if (nt == 2) {
    switch (hmax) {
      case 32: return f(integral_constant<int, 32>{}, integral_constant<int, 2>{});
      case 64: return f(integral_constant<int, 64>{}, integral_constant<int, 2>{});
      case 128: return f(integral_constant<int, 128>{}, integral_constant<int, 2>{});
      case 256: return f(integral_constant<int, 256>{}, integral_constant<int, 2>{});
    }
  } else if (nt == 3) {
    switch (hmax) {
      case 32: return f(integral_constant<int, 32>{}, integral_constant<int, 3>{});
      case 64: return f(integral_constant<int, 64>{}, integral_constant<int, 3>{});
      case 128: return f(integral_constant<int, 128>{}, integral_constant<int, 3>{});
      case 256: return f(integral_constant<int, 256>{}, integral_constant<int, 3>{});
    }
  }
  return hipErrorInvalidValue;
}

template <class K>
static hipError_t allow_lds(K kern, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_rows_bf16(const RowsArgs& A, int hmax, int nterms, hipStream_t st) {
  if (A.B <= 0) return hipSuccess;
  return dispatch_shape(hmax, nterms, [&](auto h, auto t) {
    constexpr int HMAX = decltype(h)::value, NT = decltype(t)::value;
    const int64_t waves = (A.B + 31) / 32;
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    if (A.sys.W == 1) hipLaunchKernelGGL((k_rows_bf16<HMAX, 1, NT>), dim3(blocks), dim3(256), 0, st, A);
    else hipLaunchKernelGGL((k_rows_bf16<HMAX, 2, NT>), dim3(blocks), dim3(256), 0, st, A);
    return hipGetLastError();
  });
}

// Calls f(integral_constant<NC>) for the tiles per pass `cols` if that variant is built for
// (HMAX, NT), else for the built-in one.
template <int HMAX, int NT, class F>
static hipError_t dispatch_cols(int cols, F&& f) {
  using std::integral_constant;
  if constexpr (eval_cols_available_bf16(HMAX, NT, 2) && eval_cols_default_bf16(HMAX, NT) != 2) {
    if (cols == 2) return f(integral_constant<int, 2>{});
  }
  return f(integral_constant<int, eval_cols_default_bf16(HMAX, NT)>{});
}

hipError_t launch_eval_bf16(const EvalArgs& A, int hmax, int nterms, int cols, bool ldsw, bool inplace, size_t lds,
                            unsigned grid, int waves, hipStream_t st) {
  if (A.n_items <= 0) return hipSuccess;
  return dispatch_shape(hmax, nterms, [&](auto h, auto t) {
    constexpr int HMAX = decltype(h)::value, NT = decltype(t)::value;
    return dispatch_cols<HMAX, NT>(cols, [&](auto c) {
      constexpr int NC = decltype(c)::value;
      auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        const int w = std::max(1, std::min(waves, eval_waves_bf16(HMAX, NT, NC)));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * w), lds, st, A);
        return hipGetLastError();
      };
      // in-place hidden layers where the variant is built and the network allows them
      if constexpr (inplace_kernel_bf16(HMAX, NT) && NC == 1) {
        if (inplace) {
          if (A.sys.W == 1)
            return ldsw ? go(k_eval_bf16<HMAX, 1, NT, true, true, NC>) : go(k_eval_bf16<HMAX, 1, NT, false, true, NC>);
          return ldsw ? go(k_eval_bf16<HMAX, 2, NT, true, true, NC>) : go(k_eval_bf16<HMAX, 2, NT, false, true, NC>);
        }
      }
      if (A.sys.W == 1)
        return ldsw ? go(k_eval_bf16<HMAX, 1, NT, true, false, NC>) : go(k_eval_bf16<HMAX, 1, NT, false, false, NC>);
      return ldsw ? go(k_eval_bf16<HMAX, 2, NT, true, false, NC>) : go(k_eval_bf16<HMAX, 2, NT, false, false, NC>);
    });
  });
}

hipError_t launch_eval_pauli_bf16(const EvalArgs& A, int hmax, int nterms, bool ldsw, size_t lds, unsigned grid,
                                  int waves, hipStream_t st) {
  if (A.n_items <= 0) return hipSuccess;
  if (A.sys.W != 1) return hipErrorInvalidValue;
  return dispatch_shape(hmax, nterms, [&](auto h, auto t) {
    constexpr int HMAX = decltype(h)::value, NT = decltype(t)::value;
    auto go = [&](auto kern) {
      hipError_t e = allow_lds(kern, lds);
      if (e != hipSuccess) return e;
      const int w = std::max(1, std::min(waves, eval_waves_bf16(HMAX, NT, eval_cols_default_bf16(HMAX, NT))));
      hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * w), lds, st, A);
      return hipGetLastError();
    };
    return ldsw ? go(k_eval_pauli_bf16<HMAX, NT, true>) : go(k_eval_pauli_bf16<HMAX, NT, false>);
  });
}

hipError_t launch_eval_multi_bf16(const EvalArgs* args, const int64_t* first, int n_sys, int hmax, int nterms,
                                  int cols, bool ldsw, bool inplace, size_t lds, unsigned grid, int waves,
                                  hipStream_t st) {
  return dispatch_shape(hmax, nterms, [&](auto h, auto t) {
    constexpr int HMAX = decltype(h)::value, NT = decltype(t)::value;
    return dispatch_cols<HMAX, NT>(cols, [&](auto c) {
      constexpr int NC = decltype(c)::value;
      auto go = [&](auto kern) {
        hipError_t e = allow_lds(kern, lds);
        if (e != hipSuccess) return e;
        const int w = std::max(1, std::min(waves, eval_waves_bf16(HMAX, NT, NC)));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * w), lds, st, args, first, n_sys);
        return hipGetLastError();
      };
      if constexpr (inplace_kernel_bf16(HMAX, NT) && NC == 1) {
        if (inplace)
          return ldsw ? go(k_eval_multi_bf16<HMAX, NT, true, true, NC>) : go(k_eval_multi_bf16<HMAX, NT, false, true, NC>);
      }
      return ldsw ? go(k_eval_multi_bf16<HMAX, NT, true, false, NC>) : go(k_eval_multi_bf16<HMAX, NT, false, false, NC>);
    });
  });
}

}  // namespace elocal
