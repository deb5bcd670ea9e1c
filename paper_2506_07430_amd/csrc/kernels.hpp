// Launch interfaces of the HIP kernels (host side of libelocal).
#pragma once
#include "elocal_internal.hpp"

namespace elocal {

// Offsets of the pieces of the caller's flat parameter vector.
struct ThetaLayout {
  uint32_t offW[kMaxLayers];
  uint32_t offb[kMaxLayers];
  uint32_t offwphi, offbphi, P;
};

// Arguments of the fused local-energy kernels.
struct EvalArgs {
  SysDev sys;
  MadeDev made;
  const uint64_t* x;
  int64_t B;
  const double* ediag;     // [B]
  const double* F;         // [B][nSa + nSb]
  const float* lpx;        // [B][n]   BF16 mode: log p_p(s_p) of each sample
  const double* lpx64;     // [B][n]   FP64 mode
  const double* zphi;      // [B]      phase logit of each sample
  double* partial;         // [n_items][2]
  int64_t n_items;
  uint32_t ips;            // work items per sample
  uint32_t tpi;            // row tiles per work item
  uint32_t lds_bias_off;   // byte offset of the biases in LDS (staged weights from 0)
  uint32_t lds_ctx_off;    // byte offset of the per-wave contexts
  uint32_t lds_lut_off;    // byte offset of the input-expansion table
  int32_t lds_frag[kMaxLayers];   // BF16: fragment offset of layer l's weights in LDS, or -1
                                  // when the layer is read from global memory
  // Pauli-string route only: unique flip masks [pl_len], string offsets [pl_len + 1],
  // string Z masks and real coefficients [pl_off[pl_len]]
  const uint64_t* pl_mask;
  const uint32_t* pl_off;
  const uint64_t* pl_z;
  const double* pl_coef;
  uint32_t pl_len;
};

// Arguments of the ansatz pass over the samples themselves.
struct RowsArgs {
  SysDev sys;
  MadeDev made;
  const uint64_t* x;
  int64_t B;
  float* lpx;              // [B][n] (BF16 mode)
  double* lpx64;           // [B][n] (FP64 mode)
  double* zphi;            // [B]
  double* logpsi;          // [B][2] or null
  const int64_t* count;    // if not null: only rows < min(B, *count) are evaluated (device count)
};

hipError_t launch_build_tables(int n, const double* eri, double* S, double* J2, double* K2,
                               double* J3, double* K3, hipStream_t st);
hipError_t launch_prep(const SysDev& S, const uint64_t* x, int64_t B, double* ediag, double* F,
                       hipStream_t st);
hipError_t launch_connect(const SysDev& S, const uint64_t* x, int64_t B, const double* ediag,
                          const double* F, uint64_t* xp, double* hval, int8_t* sign, uint32_t* exc,
                          hipStream_t st);
hipError_t launch_check(const SysDev& S, const uint64_t* x, int64_t B, unsigned long long* bad,
                        hipStream_t st);

// Ansatz (precision-specific): pack caller parameters, run the sample pass, run the
// fused evaluation; `hmax` is the padded hidden width class (32, 64, 128, 256).
hipError_t launch_pack_bf16(const MadeDev& M, const ThetaLayout& T, const uint16_t* theta,
                            void* frag, float* bias, hipStream_t st);
hipError_t launch_rows_bf16(const RowsArgs& A, int hmax, int nterms, hipStream_t st);
hipError_t launch_eval_bf16(const EvalArgs& A, int hmax, int nterms, int cols, bool lds_weights, bool inplace,
                            size_t lds_bytes, unsigned grid, int waves, hipStream_t st);

// Shape of the BF16 fused kernels (single and multi-system), one block per CU. A network
// pass takes NC 16-row tiles. With two fp16 terms per activation the built-in NC is 1, so
// that a wave fits in 128 registers up to width 128 (16 waves per block, four per SIMD)
// and in 256 at width 256 (8 waves, two per SIMD): the VALU and MFMA work of different
// waves on a SIMD overlap the more waves share it. NC = 2 (each weight fragment feeds
// twice the rows, in twice the registers: 8 waves per block) is also built up to width
// 128, for the autotuner. Three terms take NC = 2 (8 waves up to hmax * nterms = 256,
// else 4). A launch may use fewer waves per block than a variant is built for.
constexpr int eval_cols_default_bf16(int hmax, int nterms) { return nterms == 2 ? 1 : 2; }
constexpr bool eval_cols_available_bf16(int hmax, int nterms, int nc) {
  return nc == eval_cols_default_bf16(hmax, nterms) || (nterms == 2 && nc == 2 && hmax <= 128);
}
constexpr int eval_waves_bf16(int hmax, int nterms, int nc) {
  return nc == 1 ? (hmax <= 128 ? 16 : 8) : hmax * nterms <= 256 ? 8 : 4;
}
constexpr int kMaxEvalWavesBF16 = 16;
// Per-wave LDS context of the fused BF16 kernels: the sample's occupied/virtual lists (the
// FP64 suffix sums of its per-orbital log2 probabilities stay in registers, one per lane).
constexpr size_t kWaveCtxBytesBF16 = sizeof(SampleCtx);
// Input-expansion table of the fused BF16 kernels, in LDS after the wave contexts: entry v
// holds the 4 fp16 values (bit j of v ? 1 : 0); two entries form the layer-0 operand of 8
// input bits.
constexpr size_t kXLutBytes = 16 * 8;
// Fused BF16 kernels of at least this width do not hold the whole network in LDS: the host
// stages the layers that fit (the output layer first, then the largest others) and the
// rest is read from global memory with loads issued ahead of the products.
constexpr int kLdsPartialWidth = 256;
// LDS a fused BF16 block of `waves` waves needs beyond the staged weights and biases.
constexpr size_t block_lds_bf16(int waves) { return (size_t)waves * kWaveCtxBytesBF16 + kXLutBytes; }
// Hidden layers updated in place (INPLACE) exist for the widest two-term kernels, whose
// waves run two per SIMD in 256 registers; the host uses them when o-block pair j of every
// hidden layer reads at least j + 1 and at most j + 2 k-blocks (then one activation array
// suffices and the pair's k-loop has one runtime test). At width 128 the in-place variant
// measured 2% slower, so it is not built there.
constexpr bool inplace_kernel_bf16(int hmax, int nterms) { return hmax >= kLdsPartialWidth && nterms == 2; }
// Several systems in one launch: args[s] describes system s (device copy). BF16: system
// s owns chunks [first[s], first[s+1]) of `waves` work items each (LDS layout as
// for one system, with the bias, context and table offsets of args[0] for all). FP64:
// system s owns work items [first[s], first[s+1]).
hipError_t launch_eval_pauli_bf16(const EvalArgs& A, int hmax, int nterms, bool lds_weights, size_t lds_bytes,
                                  unsigned grid, int waves, hipStream_t st);
// Pauli route, diagonal (identity-flip) group: ediag[b] = sum_k c_k (-1)^|z_k & x_b|.
hipError_t launch_pauli_diag(const uint64_t* x, int64_t B, const uint32_t* off, const uint64_t* z,
                             const double* coef, double* ediag, hipStream_t st);
hipError_t launch_eval_multi_bf16(const EvalArgs* args, const int64_t* first, int n_sys, int hmax, int nterms,
                                  int cols, bool ldsw, bool inplace, size_t lds, unsigned grid, int waves,
                                  hipStream_t st);
hipError_t launch_eval_multi_f64(const EvalArgs* args, const int64_t* first, int n_sys, int hmax,
                                 unsigned grid, hipStream_t st);
// Host record (bytes a multiple of 4) -> device memory, in stream order.
hipError_t launch_store_bytes(const void* src, size_t bytes, void* dst, hipStream_t st);

hipError_t launch_pack_f64(const MadeDev& M, const ThetaLayout& T, const double* theta,
                           void* frag, double* bias, hipStream_t st);
hipError_t launch_rows_f64(const RowsArgs& A, int hmax, hipStream_t st);
// inplace: the two-waves-per-SIMD variant with in-place hidden layers (widths 128 and 256;
// the caller checks that the network allows it)
hipError_t launch_eval_f64(const EvalArgs& A, int hmax, bool inplace, unsigned grid, hipStream_t st);

// Sum of the per-item partials plus the diagonal: eloc[b] = ediag[b] + sum_s partial[b][s].
hipError_t launch_reduce(const double* ediag, const double* partial, int64_t B, uint32_t ips,
                         double* eloc, hipStream_t st);

// Full-sector vectors (index = rank_alpha * C(n, n_beta) + rank_beta; binom[o * 65 + i] =
// C(o, i), saturated at 2^32 - 1) and the KPM recursion on them.
hipError_t launch_sector_apply(const SysDev& S, const uint32_t* binom, int64_t dim, uint32_t nb_dim, double ch,
                               double cv, const double* v, double cz, const double* z, double* y, double* partial,
                               unsigned grid, hipStream_t st);
hipError_t launch_sector_dots(const double* partial, int64_t nw, double* dots, double* mu, int64_t n,
                              int64_t n_moments, hipStream_t st);
hipError_t launch_norm2(const double* v, int64_t dim, double* out, hipStream_t st);
hipError_t launch_sector_basis(const SysDev& S, const uint32_t* binom, int64_t dim, uint32_t nb_dim, uint64_t* x,
                               hipStream_t st);
hipError_t launch_line_shape(const double* mu, int64_t N, const double* w, int64_t P, double* rho, hipStream_t st);

// Batch-level deduplication of the connected determinants (one word per determinant).
hipError_t launch_dd_clear(uint64_t* keys, uint64_t nslots, int64_t* counters, hipStream_t st);
hipError_t launch_dd_insert(const uint64_t* xp, int64_t total, uint64_t* keys, uint64_t mask, int64_t* counters,
                            hipStream_t st);
hipError_t launch_dd_compact(const uint64_t* keys, uint64_t nslots, uint32_t* ids, uint64_t* unique, int64_t* counters,
                             hipStream_t st);
hipError_t launch_dd_assemble(const uint64_t* xp, const double* hval, int64_t B, uint32_t C, const uint64_t* keys,
                              const uint32_t* ids, uint64_t mask, const double* logpsi_u, double* eloc,
                              double* logpsi_out, int64_t* counters, hipStream_t st);

// Batch autoregressive sampling: conditional of orbital k for the first min(*Ud, cap)
// prefixes (FP64 ansatz), and one full tree step (conditionals, multinomial split of every
// prefix's weight, scan, children). The prefix count of the step is *ucur (device); the
// step writes the children's count to *unext and raises *overflow when it exceeds `cap`
// (children beyond it are not written). Launch sizes depend on `cap` only, so the steps
// need no host synchronisation.
hipError_t launch_bas_probs(const SysDev& S, const MadeDev& M, int hmax, const uint64_t* pre, const int64_t* Ud,
                            int64_t cap, int k, double* probs, hipStream_t st);
hipError_t launch_bas_step(const SysDev& S, const MadeDev& M, int hmax, const uint64_t* pre, const int64_t* w,
                           const int64_t* ucur, int64_t* unext, int64_t* overflow, int k, uint64_t seed, double* probs,
                           int64_t* counts, int64_t* off, int64_t* btot, uint64_t* child, int64_t* cw, int64_t cap,
                           hipStream_t st);
hipError_t launch_bas_root(uint64_t* pre, int64_t* w, int W, int64_t n_samples, int64_t* u0, int64_t* overflow,
                           hipStream_t st);

// Statistics and gradient (FP64).
hipError_t launch_stats(const double* eloc, const double* w, int64_t B, double* stats, hipStream_t st);

struct GradPlan {
  int n, na, nb, L;
  int dims[kMaxLayers + 1];    // 2n, widths..., 4n + 1 (phase row appended)
  ThetaLayout T;
  int precision;
  const void* theta;
  const uint64_t* x;
  const double* w;
  const double* eloc;
  int64_t B;
  double* stats;
  double* dtheta;
  // workspace pieces
  double* Wm[kMaxLayers];      // masked weights [out][in] (output layer with phase row)
  double* bm[kMaxLayers];      // biases [out]
  double* h[kMaxLayers + 1];   // activations: h[0] = bits [B][2n], h[l] [B][dims[l]], h[L+1] logits
  double* d0;                  // [B][maxdim] backward buffers
  double* d1;
  double* part;                // split-K partials: splits x part_per_split doubles
  int64_t part_per_split;
  double* dW[kMaxLayers];      // [out][in]
  double* db[kMaxLayers];      // [out]
  int splits;
};
hipError_t launch_grad(const GradPlan& G, hipStream_t st);

}  // namespace elocal
