// Internal definitions shared by the HIP translation units of libelocal.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace elocal {

typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMaxOrb = 64;
constexpr int kMaxHidden = 8;
constexpr int kMaxLayers = kMaxHidden + 1;
constexpr int kMaxOutBlocks = (4 * kMaxOrb + 1 + 15) / 16;   // 17

// Division by a fixed divisor d as a multiply and shift: q = (u * m) >> 40 with
// m = ceil(2^40 / d) is exact whenever u * d < 2^40 (here u < 2^21, d < 2^13).
struct FastDiv {
  uint32_t d;
  uint64_t m;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.m = d ? ((1ull << 40) + d - 1) / d : 0ull;
  return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t u, const FastDiv& f) {
  return (uint32_t)(((uint64_t)u * f.m) >> 40);
}

// Everything a kernel needs to know about one Hamiltonian + sector (passed by value).
struct SysDev {
  int n, na, nb, va, vb, W;
  uint32_t nSa, nSb, nDaa, nDbb, nDab;     // block sizes of the canonical list
  uint32_t npo_a, npv_a, npo_b, npv_b;     // pair counts C(m,2) of occ/vir per spin
  uint32_t C;                              // list length incl. the diagonal
  FastDiv f_va, f_vb, f_npv_a, f_npv_b, f_nSb;
  const double* h1e;                       // [n][n]
  const double* S;                         // [i][j][a][b] = (ai|bj)
  const double* J2;                        // [p][q] = (pp|qq)
  const double* K2;                        // [p][q] = (pq|qp)
  const double* J3;                        // [a][i][p] = (ai|pp)
  const double* K3;                        // [a][i][p] = (ap|pi)
  const uint16_t* pair_oa;                 // lexicographic pair k -> i | j << 8
  const uint16_t* pair_va;
  const uint16_t* pair_ob;
  const uint16_t* pair_vb;
};

// Occupied / virtual spatial-orbital lists of one determinant (per wave, in LDS).
struct SampleCtx {
  uint64_t x[2];
  uint8_t occ[2][kMaxOrb];
  uint8_t vir[2][kMaxOrb];
};

// Ansatz geometry after packing (shared by the BF16 and FP64 kernels).
//   layer l in [0, L]: l < L hidden (ReLU), l == L output: FP64 4n logits + phase row 4n;
//         BF16 4(n - 1) logits + phase row 4(n - 1) (the last orbital's conditional is 1).
//   BF16: input K split in k-blocks of 32, outputs in o-blocks of 16; one packed
//         fragment (ob, kb) = 64 lanes x 8 bf16 = 1 KiB.
//   FP64: input K split in k-steps of 4; fragment (ob, ks) = 64 lanes x 1 double.
struct MadeDev {
  int n, L;
  int nin[kMaxLayers];     // input width of layer l (true, unpadded)
  int nout[kMaxLayers];    // output width of layer l (true; output layer as above)
  int nk[kMaxLayers];      // k-blocks (BF16) or k-steps (FP64) of layer l
  int nob[kMaxLayers];     // 16-wide output blocks of layer l
  uint32_t woff[kMaxLayers];   // fragment offset of layer l in the packed buffer
  uint32_t boff[kMaxLayers];   // bias offset of layer l (padded to 16 * nob)
  uint32_t nfrag;              // total fragments
  uint32_t nbias;              // total padded biases
  // BF16 packing stores hidden units sorted by degree; o-block ob of layer l then only
  // needs its first kend[l][ob] k-blocks (the rest of its weights are masked), and only
  // those are stored: fragment kb < kend[l][ob] of o-block ob is foff[l][ob] + kb, and
  // layer l occupies fragments [foff[l][0], foff[l][nob[l]]).
  // (32-bit so that a wave-uniform lookup is a scalar load)
  int32_t kend[kMaxLayers][kMaxOutBlocks];
  int32_t foff[kMaxLayers][kMaxOutBlocks + 1];
  // BF16: kend[l][ob] again as 4-bit fields, eight per word (o-block ob in bits 4 (ob % 8)
  // of word ob / 8), so that a loop over o-blocks reads its k-ranges from three registers
  uint32_t kpack[kMaxLayers][3];
  const void* wfrag;           // packed weights (8 fp16 per lane or one double per lane)
  const void* bias;            // float (BF16 mode) or double (FP64 mode)
};

// ----------------------------------------------------------------------------- bit helpers
template <int NW>
__device__ __forceinline__ int parity_below(const uint64_t (&x)[NW], int k) {
  int c = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int lo = 64 * w;
    uint64_t m;
    if (k >= lo + 64) m = ~0ull;
    else if (k <= lo) m = 0ull;
    else m = (1ull << (k - lo)) - 1ull;
    c += __popcll(x[w] & m);
  }
  return c & 1;
}

template <int NW>
__device__ __forceinline__ void flip(uint64_t (&x)[NW], int k) {
#pragma unroll
  for (int w = 0; w < NW; ++w)
    if ((k >> 6) == w) x[w] ^= 1ull << (k & 63);
}

template <int NW>
__device__ __forceinline__ int getbit(const uint64_t (&x)[NW], int k) {
  int v = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w)
    if ((k >> 6) == w) v = (int)((x[w] >> (k & 63)) & 1ull);
  return v;
}

// Spin-orbitals below 2p that are alpha (s=0) or beta (s=1): popcount of the prefix.
template <int NW>
__device__ __forceinline__ int count_spin_below(const uint64_t (&x)[NW], int p, int s) {
  const uint64_t pat = s ? 0xAAAAAAAAAAAAAAAAull : 0x5555555555555555ull;
  const int k = 2 * p;
  int c = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int lo = 64 * w;
    uint64_t m;
    if (k >= lo + 64) m = ~0ull;
    else if (k <= lo) m = 0ull;
    else m = (1ull << (k - lo)) - 1ull;
    c += __popcll(x[w] & m & pat);
  }
  return c;
}

// First spatial orbital where two determinants differ (n if equal).
template <int NW>
__device__ __forceinline__ int first_diff_orbital(const uint64_t (&a)[NW], const uint64_t (&b)[NW], int n) {
  int k = 2 * n;
#pragma unroll
  for (int w = NW - 1; w >= 0; --w) {
    const uint64_t d = a[w] ^ b[w];
    if (d) k = 64 * w + __builtin_ctzll(d);
  }
  return k >> 1;
}

// Hidden unit at position u when the units of a layer of width w are sorted by degree
// (degree of unit j is (j mod (n-1)) + 1; ties keep ascending j). Returns -1 past w.
__host__ __device__ inline int sorted_unit(int n, int w, int u) {
  const int q = n - 1;
  for (int r = 0; r < q; ++r) {
    const int cnt = (w > r) ? (w - r - 1) / q + 1 : 0;
    if (u < cnt) return r + u * q;
    u -= cnt;
  }
  return -1;
}

// Eight occupation bits starting at bit `pos` (orbitals pos/2 .. pos/2 + 3).
template <int NW>
__device__ __forceinline__ uint32_t bits8_at(const uint64_t (&x)[NW], int pos) {
  uint64_t v = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if ((pos >> 6) == w) {
      v = x[w] >> (pos & 63);
      if (w + 1 < NW && (pos & 63) > 56) v |= x[w + 1] << (64 - (pos & 63));
    }
  }
  return (uint32_t)(v & 0xFFull);
}

// ----------------------------------------------------------------------------- the generator
// Kinds of list entries.
enum : int { KIND_DIAG = 0, KIND_SINGLE = 1, KIND_DOUBLE_SAME = 2, KIND_DOUBLE_AB = 3 };

struct Excitation {
  int kind;
  int spin;          // for singles and same-spin doubles
  uint32_t sidx;     // index of a single inside all singles (alpha then beta)
  int i, j, a, b;    // spatial orbitals (j, b unused for singles)
  int I, J, A, Bq;   // spin-orbitals (-1 unused)
};

// Unrank entry t of the canonical list of the sample in `c` (see elocal.h).
__device__ __forceinline__ Excitation unrank(const SysDev& S, const SampleCtx& c, uint32_t t) {
  Excitation e;
  e.kind = KIND_DIAG; e.spin = 0; e.sidx = 0;
  e.i = e.j = e.a = e.b = -1;
  e.I = e.J = e.A = e.Bq = -1;
  if (t == 0) return e;
  uint32_t u = t - 1;
  if (u < S.nSa) {
    e.kind = KIND_SINGLE; e.spin = 0; e.sidx = u;
    const uint32_t q = fdiv(u, S.f_va);
    e.i = c.occ[0][q]; e.a = c.vir[0][u - q * S.va];
  } else if ((u -= S.nSa) < S.nSb) {
    e.kind = KIND_SINGLE; e.spin = 1; e.sidx = S.nSa + u;
    const uint32_t q = fdiv(u, S.f_vb);
    e.i = c.occ[1][q]; e.a = c.vir[1][u - q * S.vb];
  } else if ((u -= S.nSb) < S.nDaa) {
    e.kind = KIND_DOUBLE_SAME; e.spin = 0;
    const uint32_t po = fdiv(u, S.f_npv_a), pv = u - po * S.npv_a;
    const uint16_t oo = S.pair_oa[po], vv = S.pair_va[pv];
    e.i = c.occ[0][oo & 0xFF]; e.j = c.occ[0][oo >> 8];
    e.a = c.vir[0][vv & 0xFF]; e.b = c.vir[0][vv >> 8];
  } else if ((u -= S.nDaa) < S.nDbb) {
    e.kind = KIND_DOUBLE_SAME; e.spin = 1;
    const uint32_t po = fdiv(u, S.f_npv_b), pv = u - po * S.npv_b;
    const uint16_t oo = S.pair_ob[po], vv = S.pair_vb[pv];
    e.i = c.occ[1][oo & 0xFF]; e.j = c.occ[1][oo >> 8];
    e.a = c.vir[1][vv & 0xFF]; e.b = c.vir[1][vv >> 8];
  } else {
    u -= S.nDbb;
    e.kind = KIND_DOUBLE_AB;
    const uint32_t u1 = fdiv(u, S.f_nSb), u2 = u - u1 * S.nSb;
    const uint32_t q1 = fdiv(u1, S.f_va), q2 = fdiv(u2, S.f_vb);
    e.i = c.occ[0][q1]; e.a = c.vir[0][u1 - q1 * S.va];
    e.j = c.occ[1][q2]; e.b = c.vir[1][u2 - q2 * S.vb];
  }
  if (e.kind == KIND_SINGLE) {
    e.I = 2 * e.i + e.spin; e.A = 2 * e.a + e.spin;
  } else if (e.kind == KIND_DOUBLE_SAME) {
    e.I = 2 * e.i + e.spin; e.J = 2 * e.j + e.spin; e.A = 2 * e.a + e.spin; e.Bq = 2 * e.b + e.spin;
  } else if (e.kind == KIND_DOUBLE_AB) {
    e.I = 2 * e.i; e.J = 2 * e.j + 1; e.A = 2 * e.a; e.Bq = 2 * e.b + 1;
  }
  return e;
}

// x' = a+_A a+_B a_J a_I x and the sign, operator by operator (JW parity of the prefix).
template <int NW>
__device__ __forceinline__ int apply_excitation(const uint64_t (&x)[NW], const Excitation& e,
                                                uint64_t (&xp)[NW]) {
#pragma unroll
  for (int w = 0; w < NW; ++w) xp[w] = x[w];
  if (e.kind == KIND_DIAG) return 1;
  int par = parity_below<NW>(xp, e.I);
  flip<NW>(xp, e.I);
  if (e.J >= 0) { par ^= parity_below<NW>(xp, e.J); flip<NW>(xp, e.J); }
  if (e.Bq >= 0) { par ^= parity_below<NW>(xp, e.Bq); flip<NW>(xp, e.Bq); }
  par ^= parity_below<NW>(xp, e.A);
  flip<NW>(xp, e.A);
  return par ? -1 : 1;
}

// Slater--Condon value (before the sign). Fs: this sample's single values; ed: its diagonal.
__device__ __forceinline__ double excitation_value(const SysDev& S, const Excitation& e,
                                                   const double* Fs, double ed) {
  const int n = S.n;
  switch (e.kind) {
    case KIND_DIAG: return ed;
    case KIND_SINGLE: return Fs[e.sidx];
    // 32-bit table indices: n <= 64, so n^4 < 2^25
    case KIND_DOUBLE_SAME: {
      const uint32_t nn = (uint32_t)(n * n), ab = (uint32_t)(e.a * n + e.b);
      const double d = S.S[(uint32_t)(e.i * n + e.j) * nn + ab];
      const double x = S.S[(uint32_t)(e.j * n + e.i) * nn + ab];
      return d - x;
    }
    default:
      return S.S[(uint32_t)(((e.i * n + e.j) * n + e.a) * n + e.b)];
  }
}

// Build the occupied/virtual lists of x in `c` (one wave; lane p handles orbital p).
template <int NW>
__device__ __forceinline__ void build_ctx(const SysDev& S, const uint64_t (&x)[NW], SampleCtx& c,
                                          int lane) {
  const int p = lane;
  const bool in = p < S.n;
  const bool oa = in && getbit<NW>(x, 2 * p);
  const bool ob = in && getbit<NW>(x, 2 * p + 1);
  const uint64_t ma = __ballot(oa);
  const uint64_t mb = __ballot(ob);
  const uint64_t below = (p == 0) ? 0ull : ((p >= 64) ? ~0ull : ((1ull << p) - 1ull));
  if (in) {
    const int ia = __popcll(ma & below), ib = __popcll(mb & below);
    if (oa) c.occ[0][ia] = (uint8_t)p; else c.vir[0][p - ia] = (uint8_t)p;
    if (ob) c.occ[1][ib] = (uint8_t)p; else c.vir[1][p - ib] = (uint8_t)p;
  }
#pragma unroll
  for (int w = 0; w < NW; ++w)   // static indices: x stays in registers
    if (lane == w) c.x[w] = x[w];
}

// Diagonal energy and the value of every single excitation of one sample (one wave; the
// occupied/virtual lists `c` must be visible to the whole wave):
//   E_diag = sum_p n_p h_pp + 1/2 sum_pq [n_p n_q (pp|qq) - sum_s n_ps n_qs (pq|qp)]
//   F_ai   = h_ai + sum_p n_p (ai|pp) - sum_p n_{p,s} (ap|pi)        (i -> a of spin s)
// Writes F[0 .. nSa + nSb) (single index as in the canonical list) and returns E_diag
// (the same value in every lane). Sums run in a fixed order (bitwise repeatable).
template <int NW>
__device__ __forceinline__ double sample_terms(const SysDev& S, const uint64_t (&xv)[NW], const SampleCtx& c,
                                               int lane, double* __restrict__ Fb) {
  const int n = S.n;
  double e = 0.0;
  if (lane < n) {
    const int p = lane;
    const int nap = getbit<NW>(xv, 2 * p), nbp = getbit<NW>(xv, 2 * p + 1);
    const int np_ = nap + nbp;
    if (np_) {
      double row = np_ * S.h1e[p * n + p];
      double two = 0.0;
      for (int q = 0; q < n; ++q) {
        const int naq = getbit<NW>(xv, 2 * q), nbq = getbit<NW>(xv, 2 * q + 1);
        two += (double)(np_ * (naq + nbq)) * S.J2[p * n + q] - (double)(nap * naq + nbp * nbq) * S.K2[p * n + q];
      }
      e = row + 0.5 * two;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) e += __shfl_xor(e, off);
  // singles: 8 at a time, lane = 8 * (single within the group) + (orbital residue mod 8);
  // each lane sums its residue class of orbitals (so the 8 lanes of a single read one
  // contiguous table row together), then a 3-step lane reduction
  const uint32_t nS = S.nSa + S.nSb;
  const int sub = lane >> 3, pg = lane & 7;
  for (uint32_t u0 = 0; u0 < nS; u0 += 8) {
    const uint32_t u = u0 + sub;
    const bool valid = u < nS;
    const uint32_t uu = valid ? u : 0;
    const int s = (uu < S.nSa) ? 0 : 1;
    const uint32_t v = s ? uu - S.nSa : uu;
    const int vs = s ? S.vb : S.va;
    const int i = c.occ[s][v / vs], a = c.vir[s][v % vs];
    const double* j3 = S.J3 + ((size_t)a * n + i) * n;
    const double* k3 = S.K3 + ((size_t)a * n + i) * n;
    double f = 0.0;
    for (int p = pg; p < n; p += 8) {
      const int nap = getbit<NW>(xv, 2 * p), nbp = getbit<NW>(xv, 2 * p + 1);
      f += (double)(nap + nbp) * j3[p] - (double)(s ? nbp : nap) * k3[p];
    }
    f += __shfl_xor(f, 1);
    f += __shfl_xor(f, 2);
    f += __shfl_xor(f, 4);
    if (valid && pg == 0) Fb[u] = S.h1e[a * n + i] + f;
  }
  return e;
}

}  // namespace elocal
