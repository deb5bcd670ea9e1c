// C ABI of libelocal: argument checks, workspace layout, kernel sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <cmath>
#include <utility>
#include <unordered_map>
#include <mutex>

#include "../../include/elocal.h"
#include "elocal_internal.hpp"
#include "kernels.hpp"

using namespace elocal;

namespace {

thread_local std::string g_err;

elocal_status fail(elocal_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

elocal_status hip_fail(hipError_t e, const char* what) {
  return fail(ELOCAL_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                     \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

int64_t binom2(int64_t m) { return m * (m - 1) / 2; }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Bump allocator over the caller's workspace.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? (T*)(base + off) : nullptr;
    off = align256(off + count * sizeof(T));
    return p;
  }
};

bool is_gfx950(int dev) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return false;
  return std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
}

}  // namespace

// Scratch of elocal_eval_noalloc: a file-scope device array (one copy per GPU, held until the
// process ends). Host code never passes the array's name to a kernel: each device's address
// comes from hipGetSymbolAddress, taken once per device in elocal_create with that device
// current, and is kept in g_scratch.
static constexpr size_t kNoAllocScratchBytes = (size_t)ELOCAL_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct ScratchTable {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
  hipError_t err[kMaxDevices] = {};
  bool done[kMaxDevices] = {};
};
ScratchTable& scratch_table() {
  static ScratchTable t;
  return t;
}
// Looks up this device's scratch address once (the device must be current).
void setup_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  ScratchTable& t = scratch_table();
  std::lock_guard<std::mutex> lk(t.mu);
  if (t.done[dev]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  t.ptr[dev] = (e == hipSuccess) ? p : nullptr;
  t.err[dev] = e;
  t.done[dev] = true;
}
}  // namespace

struct elocal_ctx {
  int dev = 0;
  SysDev sys{};
  double* d_h1e = nullptr;
  double* d_S = nullptr;
  double* d_J2 = nullptr;
  double* d_K2 = nullptr;
  double* d_J3 = nullptr;
  double* d_K3 = nullptr;
  uint16_t* d_pairs = nullptr;
  uint32_t* d_binom = nullptr;   // C(o, i) for o, i <= 64 (saturated), for full-sector ranks
  // Jordan--Wigner strings grouped by flip mask (elocal_pauli_build)
  uint64_t* d_pl_mask = nullptr;
  uint32_t* d_pl_off = nullptr;
  uint64_t* d_pl_z = nullptr;
  double* d_pl_coef = nullptr;
  int64_t pl_len = 0, pl_strings = 0;
  int64_t sector_dim = -1;       // C(n, n_alpha) C(n, n_beta), -1 when above 2^31 - 1
  uint32_t sector_nb = 0;        // C(n, n_beta)
  int cu_count = 256;
  // optional timing of the fused kernel
  static constexpr int kRing = 1024;
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  int64_t recorded = 0;   // pairs recorded since the last reset
  int64_t ring_pos = 0;
  // launch-shape overrides of the fused kernel (<= 0: built-in)
  int64_t tune_grid = 0;
  int64_t tune_groups = 0;
  int64_t tune_waves = 0;
  int64_t tune_cols = 0;
};

namespace {

struct AnsatzGeom {
  MadeDev md{};
  ThetaLayout T{};
  int hmax = 0;
  int precision = 0;   // storage/arithmetic family: ELOCAL_FP64 or ELOCAL_BF16
  int mode = 0;        // the caller's precision (ELOCAL_BF16X3 is in the BF16 family)
  int nterms = 2;      // fp16 terms per hidden activation (BF16 family)
  size_t wbytes = 0, bbytes = 0;
};

elocal_status make_geom(const elocal_ctx* h, const elocal_ansatz* a, AnsatzGeom& G) {
  if (!a) return fail(ELOCAL_E_INVALID, "ansatz descriptor is null");
  const int n = h->sys.n;
  if (a->n_hidden < 1 || a->n_hidden > kMaxHidden)
    return fail(ELOCAL_E_UNSUPPORTED, "n_hidden=%d outside [1, %d]", a->n_hidden, kMaxHidden);
  if (!a->widths) return fail(ELOCAL_E_INVALID, "widths is null");
  if (a->precision != ELOCAL_FP64 && a->precision != ELOCAL_BF16 && a->precision != ELOCAL_BF16X3)
    return fail(ELOCAL_E_INVALID, "precision=%d is not ELOCAL_FP64, ELOCAL_BF16 or ELOCAL_BF16X3", a->precision);
  // BF16 family: bf16 parameters on the 16-bit matrix cores; the modes differ in the number of
  // fp16 terms that carry each hidden activation
  const bool bf = a->precision != ELOCAL_FP64;
  const int L = a->n_hidden;
  int wmax = 0;
  for (int l = 0; l < L; ++l) {
    const int w = a->widths[l];
    if (w < 32 || w > 256 || w % 32)
      return fail(ELOCAL_E_UNSUPPORTED, "hidden width %d is not a multiple of 32 in [32, 256]", w);
    wmax = std::max(wmax, w);
  }
  G.hmax = wmax <= 32 ? 32 : wmax <= 64 ? 64 : wmax <= 128 ? 128 : 256;
  G.precision = bf ? ELOCAL_BF16 : ELOCAL_FP64;
  G.mode = a->precision;
  G.nterms = (a->precision == ELOCAL_BF16X3) ? 3 : 2;
  MadeDev& M = G.md;
  M.n = n;
  M.L = L;
  uint32_t wo = 0, bo = 0;
  for (int l = 0; l <= L; ++l) {
    M.nin[l] = (l == 0) ? 2 * n : a->widths[l - 1];
    // output layer: 4 logits per orbital and the phase row; the BF16 packing drops the last
    // orbital's logits (its conditional is 1) and puts the phase row in their place
    M.nout[l] = (l < L) ? a->widths[l] : bf ? 4 * (n - 1) + 1 : 4 * n + 1;
    M.nk[l] = bf ? (M.nin[l] + 31) / 32 : (M.nin[l] + 3) / 4;
    M.nob[l] = (M.nout[l] + 15) / 16;
    M.woff[l] = wo;
    M.boff[l] = bo;
    wo += (uint32_t)(M.nob[l] * M.nk[l]);
    bo += (uint32_t)(16 * M.nob[l]);
  }
  M.nfrag = wo;
  M.nbias = bo;
  // k-ranges of the degree-sorted packing: o-block ob of layer l needs the inputs of
  // degree <= the block's largest degree, a prefix of the (sorted) input order. BF16:
  // k-blocks of 32 inputs. FP64: k-steps of 4; layer 0 takes inputs 4ks..4ks+3, later
  // layers take one unit of each 4-unit group of a 16-unit block, so a prefix of units
  // is covered by whole 16-unit blocks (4 k-steps each).
  {
    auto deg_at = [&](int width, int u) { return sorted_unit(n, width, u) % (n - 1) + 1; };
    auto count_le = [&](int width, int D) {
      int c = 0;
      for (int j = 0; j < width; ++j) c += (j % (n - 1)) + 1 <= D;
      return c;
    };
    for (int l = 0; l <= L; ++l) {
      for (int ob = 0; ob < kMaxOutBlocks; ++ob) M.kend[l][ob] = M.nk[l];
      for (int ob = 0; ob < M.nob[l]; ++ob) {
        int need;   // input units (or bits) this block can see
        if (l < L) {
          const int w = a->widths[l];
          const int mmax = deg_at(w, std::min(16 * ob + 15, w - 1));
          need = (l == 0) ? 2 * mmax : count_le(a->widths[l - 1], mmax);
        } else {
          const int ph = bf ? 4 * (n - 1) : 4 * n;   // phase row
          const bool phase = 16 * ob <= ph && ph < 16 * ob + 16;
          const int D = std::min(4 * ob + 3, n - 1);
          need = phase ? M.nin[l] : count_le(a->widths[L - 1], D);
        }
        int ke;
        if (bf) ke = (need + 31) / 32;
        else ke = (l == 0) ? (need + 3) / 4 : 4 * ((need + 15) / 16);
        M.kend[l][ob] = std::min(M.nk[l], ke);
        // the BF16 kernels issue k-block 0 of every block unconditionally
        if (M.kend[l][ob] < 1) return fail(ELOCAL_E_UNSUPPORTED, "empty k-range in layer %d", l);
      }
    }
  }
  if (bf) {
    // layer 0 runs its o-blocks in pairs over one k-range, the pair's larger one (the first
    // block's extra fragments hold masked zeros); an unpaired last block is paired with a
    // phantom block of the same range
    for (int j = 0; 2 * j < M.nob[0]; ++j) {
      const int ke = 2 * j + 1 < M.nob[0] ? std::max(M.kend[0][2 * j], M.kend[0][2 * j + 1]) : M.kend[0][2 * j];
      M.kend[0][2 * j] = M.kend[0][2 * j + 1] = ke;
    }
    // compact BF16 packing: only the k-blocks each o-block uses
    uint32_t f = 0;
    for (int l = 0; l <= L; ++l) {
      for (int ob = 0; ob <= kMaxOutBlocks; ++ob) M.foff[l][ob] = 0;
      for (int ob = 0; ob < M.nob[l]; ++ob) {
        M.foff[l][ob] = (int32_t)f;
        f += (uint32_t)M.kend[l][ob];
      }
      M.foff[l][M.nob[l]] = (int32_t)f;
      M.woff[l] = (uint32_t)M.foff[l][0];
    }
    for (int l = L + 1; l < kMaxLayers; ++l)
      for (int ob = 0; ob <= kMaxOutBlocks; ++ob) M.foff[l][ob] = (int32_t)f;
    // the k-ranges as 4-bit fields (a BF16 o-block has at most 8 k-blocks)
    static_assert(kMaxOutBlocks <= 24, "three words of eight 4-bit k-ranges");
    for (int l = 0; l < kMaxLayers; ++l) {
      M.kpack[l][0] = M.kpack[l][1] = M.kpack[l][2] = 0;
      for (int ob = 0; l <= L && ob < kMaxOutBlocks; ++ob)
        M.kpack[l][ob / 8] |= (uint32_t)(M.kend[l][ob] & 15) << (4 * (ob % 8));
    }
    M.nfrag = f;
    wo = f;
  }
  G.wbytes = (size_t)wo * 64 * (bf ? 16 : 8);
  G.bbytes = (size_t)bo * (bf ? 4 : 8);
  // caller's flat layout
  uint32_t off = 0;
  for (int l = 0; l <= L; ++l) {
    const int out = (l == L) ? 4 * n : a->widths[l];
    G.T.offW[l] = off;
    off += (uint32_t)(out * M.nin[l]);
    G.T.offb[l] = off;
    off += (uint32_t)out;
  }
  G.T.offwphi = off;
  off += (uint32_t)a->widths[L - 1];
  G.T.offbphi = off;
  off += 1;
  G.T.P = off;
  return ELOCAL_OK;
}

// Work decomposition of the fused evaluation.
// LDS placement of the packed BF16 weights of one ansatz.
struct StagePlan {
  int32_t frag[kMaxLayers];   // fragment offset of layer l in LDS, -1: global memory
  size_t wbytes;              // staged weight bytes (aligned)
  bool any;                   // at least one layer staged
};

struct EvalPlan {
  uint32_t rows_per_tile, tpi, ips;
  int64_t n_items;
  bool ldsw;
  StagePlan stage;  // BF16: which layers are staged (biases follow the weights, then the
                    // wave contexts and the input table)
  bool inplace;     // hidden layers updated in place (see inplace_ok, inplace_ok_f64)
  size_t lds;
  int cols;         // BF16: 16-row tiles per network pass (kernel variant)
  int waves;        // waves per block
  unsigned grid;
};

constexpr size_t kLdsBytes = 160 * 1024;

// Persistent grid: 32 waves per CU in total (a few rounds of resident blocks), unless tuned.
int64_t grid_cap(const elocal_ctx* h, int waves) {
  if (h->tune_grid > 0) return std::min<int64_t>(h->tune_grid, 1 << 20);
  return (int64_t)h->cu_count * (32 / waves);
}

// Which layers a fused block of a width-`kernel_hmax` kernel with `waves` waves stages in
// LDS beside `bias_bytes` of biases and the wave contexts: the whole network when it fits
// (layers at their packed offsets); otherwise, from kLdsPartialWidth on, the output layer
// (read once per output block by every tile) and then the other layers, largest first,
// while they fit; below that width nothing.
static StagePlan plan_stage(const AnsatzGeom& G, int kernel_hmax, int waves, size_t bias_bytes) {
  StagePlan sp{};
  const MadeDev& M = G.md;
  for (int l = 0; l < kMaxLayers; ++l) sp.frag[l] = -1;
  const size_t fixed = align256(bias_bytes) + block_lds_bf16(waves);
  if (fixed > kLdsBytes) return sp;
  const size_t room = kLdsBytes - fixed;
  if (align256(G.wbytes) <= room) {
    for (int l = 0; l <= M.L; ++l) sp.frag[l] = M.foff[l][0];
    sp.wbytes = align256(G.wbytes);
    sp.any = true;
    return sp;
  }
  if (kernel_hmax < kLdsPartialWidth) return sp;
  int order[kMaxLayers], n = 0;
  order[n++] = M.L;
  for (int l = 0; l < M.L; ++l) order[n++] = l;
  auto frags = [&](int l) { return M.foff[l][M.nob[l]] - M.foff[l][0]; };
  std::stable_sort(order + 1, order + n, [&](int a, int b) { return frags(a) > frags(b); });
  int32_t used = 0;
  for (int i = 0; i < n; ++i) {
    const int l = order[i];
    if (align256((size_t)(used + frags(l)) * 1024) <= room) {
      sp.frag[l] = used;
      used += frags(l);
    }
  }
  sp.wbytes = align256((size_t)used * 1024);
  sp.any = used > 0;
  return sp;
}

// In-place hidden layers are exact when o-block pair j of every hidden layer reads no
// k-block beyond j + 1 (both blocks' kend <= j + 2). The in-place kernels also take both
// blocks' first j + 1 k-blocks without a test, so they need kend >= j + 1 as well (true of
// every degree-sorted network whose hidden layers have one width).
static bool inplace_ok(const MadeDev& M) {
  for (int l = 1; l < M.L; ++l)
    for (int j = 0; 2 * j < M.nob[l]; ++j) {
      const bool two = 2 * j + 1 < M.nob[l];
      const int ke = std::max(M.kend[l][2 * j], two ? M.kend[l][2 * j + 1] : 0);
      const int kl = two ? std::min(M.kend[l][2 * j], M.kend[l][2 * j + 1]) : M.kend[l][2 * j];
      if (ke > j + 2 || kl < j + 1) return false;
    }
  return true;
}

// FP64 in-place hidden layers are exact when o-block ob of every hidden layer reads no
// input block beyond ob + 1 (its k-steps, rounded up to whole chunks of 4, <= 4 (ob + 2)).
static bool inplace_ok_f64(const MadeDev& M) {
  for (int l = 1; l < M.L; ++l)
    for (int ob = 0; ob < M.nob[l]; ++ob) {
      const int kw = std::min(M.nk[l], (M.kend[l][ob] + 3) / 4 * 4);
      if (kw > 4 * (ob + 2)) return false;
    }
  return true;
}

EvalPlan plan_eval(const elocal_ctx* h, const AnsatzGeom& G, int64_t B, int64_t list_len = -1) {
  EvalPlan p{};
  // BF16: groups of 64 entries (one per lane), 8 per item; FP64: tiles of 16, 16 per item
  p.rows_per_tile = (G.precision == ELOCAL_BF16) ? 64 : 16;
  p.tpi = (G.precision == ELOCAL_BF16) ? 8 : 16;
  if (h->tune_groups > 0) p.tpi = (uint32_t)std::min<int64_t>(h->tune_groups, 1 << 16);
  // the first list entry (the sample itself) needs no ansatz call
  const uint64_t rows = (list_len > 0 ? (uint64_t)list_len : (uint64_t)h->sys.C) - 1;
  const uint64_t per_item = (uint64_t)p.rows_per_tile * p.tpi;
  p.ips = (uint32_t)((rows + per_item - 1) / per_item);
  p.n_items = (int64_t)p.ips * B;
  for (int l = 0; l < kMaxLayers; ++l) p.stage.frag[l] = -1;
  if (G.precision == ELOCAL_BF16) {
    p.cols = eval_cols_default_bf16(G.hmax, G.nterms);
    if (h->tune_cols > 0 && eval_cols_available_bf16(G.hmax, G.nterms, (int)h->tune_cols)) p.cols = (int)h->tune_cols;
    p.waves = eval_waves_bf16(G.hmax, G.nterms, p.cols);
    if (h->tune_waves > 0) p.waves = (int)std::min<int64_t>(h->tune_waves, p.waves);
    p.stage = plan_stage(G, G.hmax, p.waves, G.bbytes);
    p.ldsw = p.stage.any;   // one block per CU owns the CU's LDS
    p.lds = (p.ldsw ? p.stage.wbytes + align256(G.bbytes) : 0) + block_lds_bf16(p.waves);
    p.inplace = inplace_kernel_bf16(G.hmax, G.nterms) && p.cols == 1 && inplace_ok(G.md);
  } else {
    p.ldsw = false;
    p.lds = 0;
    p.cols = 1;
    p.waves = 4;
    p.inplace = G.hmax >= 128 && inplace_ok_f64(G.md);
  }
  const int64_t want = (p.n_items + p.waves - 1) / p.waves;
  p.grid = (unsigned)std::max<int64_t>(1, std::min(want, grid_cap(h, p.waves)));
  return p;
}

// The LDS layout fields of the BF16 kernel arguments for a plan.
void set_lds_args(EvalArgs& E, const EvalPlan& p, size_t bias_bytes) {
  const size_t wb = p.ldsw ? p.stage.wbytes : 0, bb = p.ldsw ? align256(bias_bytes) : 0;
  E.lds_bias_off = (uint32_t)wb;
  E.lds_ctx_off = (uint32_t)(wb + bb);
  E.lds_lut_off = (uint32_t)(wb + bb + (size_t)p.waves * kWaveCtxBytesBF16);
  for (int l = 0; l < kMaxLayers; ++l) E.lds_frag[l] = p.ldsw ? p.stage.frag[l] : -1;
}

struct EvalWs {
  double* ediag;
  double* F;
  void* frag;
  void* bias;
  float* lpx;
  double* lpx64;
  double* zphi;
  double* partial;
  size_t bytes;
};

EvalWs carve_eval(const elocal_ctx* h, const AnsatzGeom& G, const EvalPlan& p, int64_t B, void* ws) {
  Carve c(ws);
  EvalWs w{};
  const size_t nS = h->sys.nSa + h->sys.nSb;
  w.ediag = c.take<double>(std::max<int64_t>(B, 1));
  w.F = c.take<double>(std::max<size_t>((size_t)B * nS, 1));
  w.frag = c.take<char>(G.wbytes);
  w.bias = c.take<char>(G.bbytes);
  if (G.precision == ELOCAL_BF16) {
    w.lpx = c.take<float>(std::max<size_t>((size_t)B * h->sys.n, 1));
    w.lpx64 = nullptr;
  } else {
    w.lpx = nullptr;
    w.lpx64 = c.take<double>(std::max<size_t>((size_t)B * h->sys.n, 1));
  }
  w.zphi = c.take<double>(std::max<int64_t>(B, 1));
  w.partial = c.take<double>(std::max<size_t>((size_t)p.n_items * 2, 1));
  w.bytes = c.off;
  return w;
}

struct ConnectWs {
  double* ediag;
  double* F;
  size_t bytes;
};

ConnectWs carve_connect(const elocal_ctx* h, int64_t B, void* ws) {
  Carve c(ws);
  ConnectWs w{};
  const size_t nS = h->sys.nSa + h->sys.nSb;
  w.ediag = c.take<double>(std::max<int64_t>(B, 1));
  w.F = c.take<double>(std::max<size_t>((size_t)B * nS, 1));
  w.bytes = c.off;
  return w;
}

size_t carve_grad(const elocal_ctx* h, const AnsatzGeom& G, int64_t B, void* ws, GradPlan* out) {
  Carve c(ws);
  GradPlan P{};
  const int L = G.md.L, n = h->sys.n;
  P.n = n; P.na = h->sys.na; P.nb = h->sys.nb; P.L = L;
  P.dims[0] = 2 * n;
  for (int l = 0; l < L; ++l) P.dims[l + 1] = G.md.nout[l];
  P.dims[L + 1] = 4 * n + 1;
  int maxdim = 0;
  size_t maxw = 0;
  for (int l = 0; l <= L + 1; ++l) maxdim = std::max(maxdim, P.dims[l]);
  for (int l = 0; l <= L; ++l) {
    const size_t cnt = (size_t)P.dims[l + 1] * P.dims[l];
    maxw = std::max(maxw, cnt);
    P.Wm[l] = c.take<double>(cnt);
    P.bm[l] = c.take<double>(P.dims[l + 1]);
    P.dW[l] = c.take<double>(cnt);
    P.db[l] = c.take<double>(P.dims[l + 1]);
  }
  const size_t Bs = (size_t)std::max<int64_t>(B, 1);
  for (int l = 0; l <= L + 1; ++l) P.h[l] = c.take<double>(Bs * P.dims[l]);
  P.d0 = c.take<double>(Bs * maxdim);
  P.d1 = c.take<double>(Bs * maxdim);
  P.splits = (int)std::min<int64_t>(64, std::max<int64_t>(1, B / 256));
  P.part = c.take<double>((size_t)P.splits * maxw);
  P.part_per_split = (int64_t)maxw;
  P.T = G.T;
  P.precision = G.precision;
  if (out) *out = P;
  return c.off;
}

SysDev build_sys(int n, int na, int nb) {
  SysDev s{};
  s.n = n; s.na = na; s.nb = nb; s.va = n - na; s.vb = n - nb;
  s.W = (2 * n + 63) / 64;
  s.nSa = (uint32_t)(na * s.va);
  s.nSb = (uint32_t)(nb * s.vb);
  s.npo_a = (uint32_t)binom2(na); s.npv_a = (uint32_t)binom2(s.va);
  s.npo_b = (uint32_t)binom2(nb); s.npv_b = (uint32_t)binom2(s.vb);
  s.nDaa = s.npo_a * s.npv_a;
  s.nDbb = s.npo_b * s.npv_b;
  s.nDab = s.nSa * s.nSb;
  s.C = 1u + s.nSa + s.nSb + s.nDaa + s.nDbb + s.nDab;
  s.f_va = make_fastdiv((uint32_t)s.va);
  s.f_vb = make_fastdiv((uint32_t)s.vb);
  s.f_npv_a = make_fastdiv(s.npv_a);
  s.f_npv_b = make_fastdiv(s.npv_b);
  s.f_nSb = make_fastdiv(s.nSb);
  return s;
}

elocal_status check_device(const elocal_ctx* h) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != h->dev) return fail(ELOCAL_E_DEVICE, "current device %d is not the handle's device %d", dev, h->dev);
  return ELOCAL_OK;
}

}  // namespace

extern "C" {

const char* elocal_last_error(void) { return g_err.c_str(); }

int64_t elocal_num_params(int n_orb, int n_hidden, const int* widths) {
  if (n_orb < 2 || n_orb > kMaxOrb || n_hidden < 1 || n_hidden > kMaxHidden || !widths) return -1;
  int64_t p = 0;
  int in = 2 * n_orb;
  for (int l = 0; l < n_hidden; ++l) {
    if (widths[l] < 1) return -1;
    p += (int64_t)widths[l] * in + widths[l];
    in = widths[l];
  }
  p += (int64_t)4 * n_orb * in + 4 * n_orb;
  p += in + 1;
  return p;
}

elocal_status elocal_create(const double* h1e, const double* eri, int n_orb, int n_alpha, int n_beta,
                            elocal_t* out) {
  if (!out) return fail(ELOCAL_E_INVALID, "out is null");
  *out = nullptr;
  if (!h1e || !eri) return fail(ELOCAL_E_INVALID, "h1e or eri is null");
  if (n_orb < 2 || n_orb > kMaxOrb) return fail(ELOCAL_E_UNSUPPORTED, "n_orb=%d outside [2, %d]", n_orb, kMaxOrb);
  if (n_alpha < 0 || n_beta < 0 || n_alpha > n_orb || n_beta > n_orb)
    return fail(ELOCAL_E_INVALID, "electron counts (%d, %d) outside [0, n_orb=%d]", n_alpha, n_beta, n_orb);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) return fail(ELOCAL_E_DEVICE, "no HIP device available");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (!is_gfx950(dev)) return fail(ELOCAL_E_DEVICE, "device %d is not gfx950", dev);
  setup_scratch(dev);
  elocal_ctx* h = new elocal_ctx();
  h->dev = dev;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      h->cu_count = prop.multiProcessorCount;
  }
  h->sys = build_sys(n_orb, n_alpha, n_beta);
  const size_t n = n_orb, n2 = n * n, n3 = n2 * n, n4 = n3 * n;
  // pair tables for m = n_alpha, n - n_alpha, n_beta, n - n_beta
  const int ms[4] = {n_alpha, n_orb - n_alpha, n_beta, n_orb - n_beta};
  std::vector<uint16_t> pairs;
  size_t poff[4];
  for (int t = 0; t < 4; ++t) {
    poff[t] = pairs.size();
    for (int i = 0; i < ms[t]; ++i)
      for (int j = i + 1; j < ms[t]; ++j) pairs.push_back((uint16_t)(i | (j << 8)));
  }
  if (pairs.empty()) pairs.push_back(0);
  std::vector<uint32_t> binom(65 * 65, 0);
  for (int o = 0; o <= 64; ++o) {
    uint64_t c = 1;   // C(o, 0); then C(o, i) = C(o, i - 1) (o - i + 1) / i, exact while small
    bool big = false;
    for (int i = 0; i <= 64; ++i) {
      if (i > 0) {
        if (i > o) c = 0;
        else if (!big) {
          const unsigned __int128 t = (unsigned __int128)c * (uint64_t)(o - i + 1);
          c = (uint64_t)(t / (uint64_t)i);
          big = c > 0xFFFFFFFFull;
        }
      }
      binom[o * 65 + i] = (i > o) ? 0u : (big ? 0xFFFFFFFFu : (uint32_t)c);
    }
  }
  double* d_eri = nullptr;
  auto cleanup = [&](elocal_status st) {
    hipFree(d_eri);
    hipFree(h->d_h1e); hipFree(h->d_S); hipFree(h->d_J2); hipFree(h->d_K2);
    hipFree(h->d_J3); hipFree(h->d_K3); hipFree(h->d_pairs); hipFree(h->d_binom);
  hipFree(h->d_pl_mask); hipFree(h->d_pl_off); hipFree(h->d_pl_z); hipFree(h->d_pl_coef);
    delete h;
    return st;
  };
  if (hipMalloc(&h->d_h1e, n2 * 8) != hipSuccess || hipMalloc(&d_eri, n4 * 8) != hipSuccess ||
      hipMalloc(&h->d_S, n4 * 8) != hipSuccess || hipMalloc(&h->d_J2, n2 * 8) != hipSuccess ||
      hipMalloc(&h->d_K2, n2 * 8) != hipSuccess || hipMalloc(&h->d_J3, n3 * 8) != hipSuccess ||
      hipMalloc(&h->d_K3, n3 * 8) != hipSuccess ||
      hipMalloc(&h->d_pairs, pairs.size() * sizeof(uint16_t)) != hipSuccess ||
      hipMalloc(&h->d_binom, binom.size() * sizeof(uint32_t)) != hipSuccess)
    return cleanup(fail(ELOCAL_E_NOMEM, "device allocation failed in elocal_create"));
  hipError_t err = hipMemcpy(h->d_h1e, h1e, n2 * 8, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(d_eri, eri, n4 * 8, hipMemcpyHostToDevice);
  if (err == hipSuccess)
    err = hipMemcpy(h->d_pairs, pairs.data(), pairs.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  if (err == hipSuccess)
    err = hipMemcpy(h->d_binom, binom.data(), binom.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = launch_build_tables(n_orb, d_eri, h->d_S, h->d_J2, h->d_K2, h->d_J3, h->d_K3, nullptr);
  if (err == hipSuccess) err = hipDeviceSynchronize();
  if (err != hipSuccess) return cleanup(hip_fail(err, "elocal_create"));
  hipFree(d_eri);
  d_eri = nullptr;
  SysDev& s = h->sys;
  s.h1e = h->d_h1e; s.S = h->d_S; s.J2 = h->d_J2; s.K2 = h->d_K2; s.J3 = h->d_J3; s.K3 = h->d_K3;
  s.pair_oa = h->d_pairs + poff[0];
  s.pair_va = h->d_pairs + poff[1];
  s.pair_ob = h->d_pairs + poff[2];
  s.pair_vb = h->d_pairs + poff[3];
  {
    const uint64_t ca = binom[n_orb * 65 + n_alpha], cb = binom[n_orb * 65 + n_beta];
    const bool fits = ca < 0xFFFFFFFFull && cb < 0xFFFFFFFFull && ca * cb <= 0x7FFFFFFFull;
    h->sector_dim = fits ? (int64_t)(ca * cb) : -1;
    h->sector_nb = (uint32_t)cb;
  }
  *out = h;
  return ELOCAL_OK;
}

elocal_status elocal_destroy(elocal_t h) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  for (hipEvent_t e : h->ev_start) hipEventDestroy(e);
  for (hipEvent_t e : h->ev_stop) hipEventDestroy(e);
  hipFree(h->d_h1e); hipFree(h->d_S); hipFree(h->d_J2); hipFree(h->d_K2);
  hipFree(h->d_J3); hipFree(h->d_K3); hipFree(h->d_pairs); hipFree(h->d_binom);
  hipFree(h->d_pl_mask); hipFree(h->d_pl_off); hipFree(h->d_pl_z); hipFree(h->d_pl_coef);
  delete h;
  return ELOCAL_OK;
}

int64_t elocal_num_connected(elocal_t h) { return h ? (int64_t)h->sys.C : -1; }

int elocal_words(elocal_t h) { return h ? h->sys.W : -1; }

size_t elocal_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t B, int op) {
  if (!h) { fail(ELOCAL_E_INVALID, "handle is null"); return 0; }
  if (B < 0) { fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B); return 0; }
  if (op == ELOCAL_OP_CONNECT) return carve_connect(h, B, nullptr).bytes;
  AnsatzGeom G;
  if (make_geom(h, a, G) != ELOCAL_OK) return 0;
  if (op == ELOCAL_OP_EVAL) {
    const EvalPlan p = plan_eval(h, G, B);
    return carve_eval(h, G, p, B, nullptr).bytes;
  }
  if (op == ELOCAL_OP_GRAD) return carve_grad(h, G, B, nullptr, nullptr);
  fail(ELOCAL_E_INVALID, "unknown op %d", op);
  return 0;
}

elocal_status elocal_connect(elocal_t h, elocal_stream s, const uint64_t* x, int64_t B, void* ws,
                             size_t ws_bytes, uint64_t* xp, double* hval, int8_t* sign, uint32_t* exc) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (B < 0) return fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B);
  if (B == 0) return ELOCAL_OK;
  if (!x || !ws || !xp || !hval || !sign || !exc) return fail(ELOCAL_E_INVALID, "null pointer argument");
  const ConnectWs need = carve_connect(h, B, nullptr);
  if (ws_bytes < need.bytes)
    return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need.bytes);
  if (elocal_status st = check_device(h)) return st;
  const ConnectWs w = carve_connect(h, B, ws);
  hipStream_t st = (hipStream_t)s;
  HIP_TRY(launch_prep(h->sys, x, B, w.ediag, w.F, st), "prep launch");
  const int slot = (int)(h->ring_pos % elocal_ctx::kRing);
  if (h->timing) HIP_TRY(hipEventRecord(h->ev_start[slot], st), "timing event");
  HIP_TRY(launch_connect(h->sys, x, B, w.ediag, w.F, xp, hval, sign, exc, st), "connect launch");
  if (h->timing) {
    HIP_TRY(hipEventRecord(h->ev_stop[slot], st), "timing event");
    h->ring_pos++;
    h->recorded++;
  }
  return ELOCAL_OK;
}

elocal_status elocal_eval(elocal_t h, elocal_stream s, const elocal_ansatz* a, const uint64_t* x, int64_t B,
                          void* ws, size_t ws_bytes, double* eloc, double* logpsi) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  AnsatzGeom G;
  if (elocal_status e = make_geom(h, a, G)) return e;
  if (B < 0) return fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B);
  if (B == 0) return ELOCAL_OK;
  if (!a->theta || !x || !ws || !eloc) return fail(ELOCAL_E_INVALID, "null pointer argument");
  const EvalPlan p = plan_eval(h, G, B);
  const EvalWs need = carve_eval(h, G, p, B, nullptr);
  if (ws_bytes < need.bytes)
    return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need.bytes);
  if (elocal_status st = check_device(h)) return st;
  const EvalWs w = carve_eval(h, G, p, B, ws);
  hipStream_t st = (hipStream_t)s;
  MadeDev M = G.md;
  M.wfrag = w.frag;
  M.bias = w.bias;
  if (G.precision == ELOCAL_BF16)
    HIP_TRY(launch_pack_bf16(M, G.T, (const uint16_t*)a->theta, w.frag, (float*)w.bias, st), "pack launch");
  else
    HIP_TRY(launch_pack_f64(M, G.T, (const double*)a->theta, w.frag, (double*)w.bias, st), "pack launch");
  HIP_TRY(launch_prep(h->sys, x, B, w.ediag, w.F, st), "prep launch");
  RowsArgs R{};
  R.sys = h->sys; R.made = M; R.x = x; R.B = B; R.lpx = w.lpx; R.lpx64 = w.lpx64; R.zphi = w.zphi;
  R.logpsi = logpsi;
  if (G.precision == ELOCAL_BF16) HIP_TRY(launch_rows_bf16(R, G.hmax, G.nterms, st), "sample pass launch");
  else HIP_TRY(launch_rows_f64(R, G.hmax, st), "sample pass launch");
  EvalArgs E{};
  E.sys = h->sys; E.made = M; E.x = x; E.B = B; E.ediag = w.ediag; E.F = w.F; E.lpx = w.lpx;
  E.lpx64 = w.lpx64; E.zphi = w.zphi; E.partial = w.partial; E.n_items = p.n_items; E.ips = p.ips;
  E.tpi = p.tpi;
  const bool timed = h->timing && p.n_items > 0;
  const int slot = (int)(h->ring_pos % elocal_ctx::kRing);
  if (timed) HIP_TRY(hipEventRecord(h->ev_start[slot], st), "timing event");
  if (G.precision == ELOCAL_BF16) {
    set_lds_args(E, p, G.bbytes);
    HIP_TRY(launch_eval_bf16(E, G.hmax, G.nterms, p.cols, p.ldsw, p.inplace, p.lds, p.grid, p.waves, st),
            "eval launch");
  } else {
    HIP_TRY(launch_eval_f64(E, G.hmax, p.inplace, p.grid, st), "eval launch");
  }
  if (timed) {
    HIP_TRY(hipEventRecord(h->ev_stop[slot], st), "timing event");
    h->ring_pos++;
    h->recorded++;
  }
  HIP_TRY(launch_reduce(w.ediag, w.partial, B, p.ips, eloc, st), "reduce launch");
  return ELOCAL_OK;
}

elocal_status elocal_eval_noalloc(elocal_t h, elocal_stream s, const elocal_ansatz* a, const uint64_t* x,
                                  int64_t B, double* eloc, double* logpsi) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (elocal_status st = check_device(h)) return st;
  void* ws = nullptr;
  {
    ScratchTable& t = scratch_table();
    std::lock_guard<std::mutex> lk(t.mu);
    if (h->dev < 0 || h->dev >= kMaxDevices || !t.done[h->dev])
      return fail(ELOCAL_E_DEVICE, "no scratch address for device %d", h->dev);
    if (!t.ptr[h->dev]) return hip_fail(t.err[h->dev], "hipGetSymbolAddress(scratch)");
    ws = t.ptr[h->dev];
  }
  AnsatzGeom G;
  if (elocal_status e = make_geom(h, a, G)) return e;
  if (B < 0) return fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B);
  const size_t need = carve_eval(h, G, plan_eval(h, G, B), B, nullptr).bytes;
  if (need > kNoAllocScratchBytes)
    return fail(ELOCAL_E_WORKSPACE,
                "elocal_eval_noalloc needs %zu bytes of scratch for B=%lld, above its fixed %zu bytes "
                "(ELOCAL_NOALLOC_SCRATCH_MIB); use elocal_eval with a caller workspace or a smaller batch",
                need, (long long)B, kNoAllocScratchBytes);
  return elocal_eval(h, s, a, x, B, ws, kNoAllocScratchBytes, eloc, logpsi);
}

namespace {

// Layout and launch plan of elocal_eval_multi: per-system eval workspaces back to back,
// then the device copies of the per-system kernel arguments and the item prefix.
struct MultiPlan {
  AnsatzGeom G[ELOCAL_MAX_SYSTEMS];
  EvalPlan p[ELOCAL_MAX_SYSTEMS];
  size_t off[ELOCAL_MAX_SYSTEMS];   // byte offset of system s's eval workspace
  int order[ELOCAL_MAX_SYSTEMS];    // position in the item space -> system
  size_t args_off, first_off, bytes;
  int64_t first[ELOCAL_MAX_SYSTEMS + 1];
  int hmax, precision;
  bool ldsw;            // BF16: some system stages weights in LDS
  bool inplace;         // BF16: in-place hidden layers (every system allows them)
  int cols, waves;      // BF16: tiles per pass and waves per block of the launch
  StagePlan stage[ELOCAL_MAX_SYSTEMS];   // BF16: system s's staged layers
  uint32_t bias_off, ctx_off, lut_off;   // BF16: the LDS layout every system shares
  size_t lds;
  unsigned grid;
};

// the kernels index a plain array EvalArgs[n_sys]
constexpr size_t kArgsStride = sizeof(EvalArgs);
static_assert(sizeof(EvalArgs) % 8 == 0, "EvalArgs is stored in 4-byte words");

elocal_status plan_multi(int n_sys, const elocal_t* hs, const elocal_ansatz* const* a, const int64_t* B,
                         MultiPlan& M) {
  if (n_sys < 1 || n_sys > ELOCAL_MAX_SYSTEMS)
    return fail(ELOCAL_E_INVALID, "n_sys=%d outside [1, %d]", n_sys, (int)ELOCAL_MAX_SYSTEMS);
  if (!hs || !a || !B) return fail(ELOCAL_E_INVALID, "null array argument");
  M.hmax = 0;
  size_t off = 0;
  double cost[ELOCAL_MAX_SYSTEMS];
  for (int s = 0; s < n_sys; ++s) {
    if (!hs[s]) return fail(ELOCAL_E_INVALID, "handle %d is null", s);
    if (hs[s]->dev != hs[0]->dev) return fail(ELOCAL_E_INVALID, "handles %d and 0 are on different devices", s);
    if (B[s] < 0) return fail(ELOCAL_E_INVALID, "B[%d]=%lld is negative", s, (long long)B[s]);
    if (elocal_status e = make_geom(hs[s], a[s], M.G[s])) return e;
    if (s > 0 && M.G[s].mode != M.G[0].mode)
      return fail(ELOCAL_E_INVALID, "ansatz %d has another precision than ansatz 0", s);
    M.hmax = std::max(M.hmax, M.G[s].hmax);
    M.p[s] = plan_eval(hs[s], M.G[s], B[s]);
    M.off[s] = off;
    off = align256(off + carve_eval(hs[s], M.G[s], M.p[s], B[s], nullptr).bytes);
    // cost of one item ~ rows x dense multiply-adds per row
    double per_row = 0.0;
    const MadeDev& md = M.G[s].md;
    for (int l = 0; l <= md.L; ++l) per_row += (double)md.nin[l] * md.nout[l];
    cost[s] = per_row * M.p[s].rows_per_tile * M.p[s].tpi;
    M.order[s] = s;
  }
  M.precision = M.G[0].precision;
  // most expensive items first: the grid's last items are then the cheapest ones
  std::stable_sort(M.order, M.order + n_sys, [&](int u, int v) { return cost[u] > cost[v]; });
  // BF16: index space of chunks (one item per wave of a block, never two systems in a
  // chunk); FP64: index space of items
  // BF16 launch shape: the first handle's tuning, for the widest system's kernel
  M.cols = eval_cols_default_bf16(M.hmax, M.G[0].nterms);
  if (hs[0]->tune_cols > 0 && eval_cols_available_bf16(M.hmax, M.G[0].nterms, (int)hs[0]->tune_cols))
    M.cols = (int)hs[0]->tune_cols;
  M.waves = eval_waves_bf16(M.hmax, M.G[0].nterms, M.cols);
  if (hs[0]->tune_waves > 0) M.waves = (int)std::min<int64_t>(hs[0]->tune_waves, M.waves);
  const int unit = (M.precision == ELOCAL_BF16) ? M.waves : 1;
  M.first[0] = 0;
  for (int i = 0; i < n_sys; ++i) M.first[i + 1] = M.first[i] + (M.p[M.order[i]].n_items + unit - 1) / unit;
  M.ldsw = M.inplace = false;
  M.bias_off = M.ctx_off = M.lut_off = 0;
  M.lds = 0;
  if (M.precision == ELOCAL_BF16) {
    // one LDS layout for all systems, sized for the kernel's width class and wave count
    const int waves = M.waves;
    size_t wmax = 0, bmax = 0;
    for (int s = 0; s < n_sys; ++s) bmax = std::max(bmax, align256(M.G[s].bbytes));
    M.inplace = inplace_kernel_bf16(M.hmax, M.G[0].nterms) && M.cols == 1;
    for (int s = 0; s < n_sys; ++s) {
      M.stage[s] = plan_stage(M.G[s], M.hmax, waves, bmax);
      M.ldsw = M.ldsw || M.stage[s].any;
      wmax = std::max(wmax, M.stage[s].wbytes);
      M.inplace = M.inplace && inplace_ok(M.G[s].md);
    }
    if (M.ldsw) {
      M.bias_off = (uint32_t)wmax;
      M.ctx_off = (uint32_t)(wmax + bmax);
    }
    M.lut_off = M.ctx_off + (uint32_t)((size_t)waves * kWaveCtxBytesBF16);
    M.lds = M.ctx_off + block_lds_bf16(waves);
  }
  M.args_off = off;
  off = align256(off + kArgsStride * n_sys);
  M.first_off = off;
  off = align256(off + sizeof(int64_t) * (n_sys + 1));
  M.bytes = off;
  const int waves = (M.precision == ELOCAL_BF16) ? M.waves : 4;
  const int64_t want = (M.precision == ELOCAL_BF16) ? M.first[n_sys] : (M.first[n_sys] + 3) / 4;
  M.grid = (unsigned)std::max<int64_t>(1, std::min(want, grid_cap(hs[0], waves)));
  return ELOCAL_OK;
}

}  // namespace

size_t elocal_workspace_bytes_multi(int n_sys, const elocal_t* hs, const elocal_ansatz* const* a,
                                    const int64_t* B) {
  MultiPlan M;
  if (plan_multi(n_sys, hs, a, B, M) != ELOCAL_OK) return 0;
  return M.bytes;
}

elocal_status elocal_eval_multi(int n_sys, const elocal_t* hs, elocal_stream s, const elocal_ansatz* const* a,
                                const uint64_t* const* x, const int64_t* B, void* ws, size_t ws_bytes,
                                double* const* eloc, double* const* logpsi) {
  MultiPlan M;
  if (elocal_status e = plan_multi(n_sys, hs, a, B, M)) return e;
  if (!x || !eloc) return fail(ELOCAL_E_INVALID, "null array argument");
  if (!ws) return fail(ELOCAL_E_INVALID, "workspace is null");
  for (int i = 0; i < n_sys; ++i)
    if (B[i] > 0 && (!a[i]->theta || !x[i] || !eloc[i])) return fail(ELOCAL_E_INVALID, "null pointer for system %d", i);
  if (ws_bytes < M.bytes) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, M.bytes);
  if (elocal_status st = check_device(hs[0])) return st;
  hipStream_t st = (hipStream_t)s;
  char* base = (char*)ws;
  EvalArgs* d_args = (EvalArgs*)(base + M.args_off);
  int64_t* d_first = (int64_t*)(base + M.first_off);
  EvalWs W[ELOCAL_MAX_SYSTEMS];
  // per-system sample passes (packing, diagonal/Fock terms, ansatz at the samples)
  for (int i = 0; i < n_sys; ++i) {
    const elocal_ctx* h = hs[i];
    const AnsatzGeom& G = M.G[i];
    W[i] = carve_eval(h, G, M.p[i], B[i], base + M.off[i]);
    if (B[i] == 0) continue;
    MadeDev md = G.md;
    md.wfrag = W[i].frag;
    md.bias = W[i].bias;
    if (G.precision == ELOCAL_BF16)
      HIP_TRY(launch_pack_bf16(md, G.T, (const uint16_t*)a[i]->theta, W[i].frag, (float*)W[i].bias, st), "pack launch");
    else
      HIP_TRY(launch_pack_f64(md, G.T, (const double*)a[i]->theta, W[i].frag, (double*)W[i].bias, st), "pack launch");
    HIP_TRY(launch_prep(h->sys, x[i], B[i], W[i].ediag, W[i].F, st), "prep launch");
    RowsArgs R{};
    R.sys = h->sys; R.made = md; R.x = x[i]; R.B = B[i]; R.lpx = W[i].lpx; R.lpx64 = W[i].lpx64;
    R.zphi = W[i].zphi; R.logpsi = logpsi ? logpsi[i] : nullptr;
    if (G.precision == ELOCAL_BF16) HIP_TRY(launch_rows_bf16(R, G.hmax, G.nterms, st), "sample pass launch");
    else HIP_TRY(launch_rows_f64(R, G.hmax, st), "sample pass launch");
  }
  // kernel arguments of every system, in item-space order, and the item prefix
  for (int k = 0; k < n_sys; ++k) {
    const int i = M.order[k];
    const elocal_ctx* h = hs[i];
    EvalArgs E{};
    E.sys = h->sys; E.made = M.G[i].md; E.made.wfrag = W[i].frag; E.made.bias = W[i].bias;
    E.x = x[i]; E.B = B[i]; E.ediag = W[i].ediag; E.F = W[i].F; E.lpx = W[i].lpx; E.lpx64 = W[i].lpx64;
    E.zphi = W[i].zphi; E.partial = W[i].partial; E.n_items = M.p[i].n_items; E.ips = M.p[i].ips;
    E.tpi = M.p[i].tpi; E.lds_bias_off = M.bias_off; E.lds_ctx_off = M.ctx_off; E.lds_lut_off = M.lut_off;
    for (int l = 0; l < kMaxLayers; ++l) E.lds_frag[l] = M.ldsw ? M.stage[i].frag[l] : -1;
    HIP_TRY(launch_store_bytes(&E, sizeof(EvalArgs), (char*)d_args + kArgsStride * k, st), "argument store");
  }
  HIP_TRY(launch_store_bytes(M.first, sizeof(int64_t) * (n_sys + 1), d_first, st), "argument store");
  elocal_ctx* h0 = hs[0];
  const bool timed = h0->timing && M.first[n_sys] > 0;
  const int slot = (int)(h0->ring_pos % elocal_ctx::kRing);
  if (M.first[n_sys] > 0) {
    if (timed) HIP_TRY(hipEventRecord(h0->ev_start[slot], st), "timing event");
    if (M.precision == ELOCAL_BF16)
      HIP_TRY(launch_eval_multi_bf16(d_args, d_first, n_sys, M.hmax, M.G[0].nterms, M.cols, M.ldsw, M.inplace, M.lds,
                                     M.grid, M.waves, st),
              "multi eval launch");
    else
      HIP_TRY(launch_eval_multi_f64(d_args, d_first, n_sys, M.hmax, M.grid, st), "multi eval launch");
    if (timed) {
      HIP_TRY(hipEventRecord(h0->ev_stop[slot], st), "timing event");
      h0->ring_pos++;
      h0->recorded++;
    }
  }
  for (int i = 0; i < n_sys; ++i)
    if (B[i] > 0) HIP_TRY(launch_reduce(W[i].ediag, W[i].partial, B[i], M.p[i].ips, eloc[i], st), "reduce launch");
  return ELOCAL_OK;
}

// ----------------------------------------------------------------------------- Pauli strings
namespace {

// A Pauli string on 2n <= 64 qubits as c X^x Z^z (on every qubit X before Z), so that
// (X^x1 Z^z1)(X^x2 Z^z2) = (-1)^|z1 & x2| X^(x1^x2) Z^(z1^z2). With Y = i X Z the
// ladder operators of the Jordan--Wigner map are real:
//   a+_j = Z_{<j} (X_j - i Y_j) / 2 = (X_j + X_j Z_j) Z_{<j} / 2,
//   a_j  = Z_{<j} (X_j + i Y_j) / 2 = (X_j - X_j Z_j) Z_{<j} / 2.
struct PTerm {
  double c;
  uint64_t x, z;
};

void ladder(int j, bool dagger, PTerm out[2]) {
  const uint64_t e = 1ull << j, zs = e - 1;
  out[0] = {0.5, e, zs};
  out[1] = {dagger ? 0.5 : -0.5, e, zs | e};
}

struct KeyHash {
  size_t operator()(const std::pair<uint64_t, uint64_t>& k) const {
    return std::hash<uint64_t>()(k.first * 0x9E3779B97F4A7C15ull ^ (k.second + 0x632BE59BD9B4E019ull));
  }
};

// coefficient map of sum_ops coef * (product of the ladder operators), accumulated
void add_product(std::unordered_map<std::pair<uint64_t, uint64_t>, double, KeyHash>& acc, double coef,
                 const int* modes, const bool* dag, int k) {
  PTerm terms[16];
  int nt = 1;
  terms[0] = {coef, 0, 0};
  for (int o = 0; o < k; ++o) {
    PTerm l[2];
    ladder(modes[o], dag[o], l);
    PTerm next[16];
    int m = 0;
    for (int a = 0; a < nt; ++a)
      for (int b = 0; b < 2; ++b) {
        const int sgn = (__builtin_popcountll(terms[a].z & l[b].x) & 1) ? -1 : 1;
        next[m++] = {terms[a].c * l[b].c * sgn, terms[a].x ^ l[b].x, terms[a].z ^ l[b].z};
      }
    nt = m;
    for (int a = 0; a < nt; ++a) terms[a] = next[a];
  }
  for (int a = 0; a < nt; ++a) acc[{terms[a].x, terms[a].z}] += terms[a].c;
}

}  // namespace

elocal_status elocal_pauli_build(elocal_t h, const double* h1e, const double* eri) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (!h1e || !eri) return fail(ELOCAL_E_INVALID, "h1e or eri is null");
  const int n = h->sys.n;
  if (2 * n > 64) return fail(ELOCAL_E_UNSUPPORTED, "the Pauli route needs 2 n <= 64 (n=%d)", n);
  if (elocal_status st = check_device(h)) return st;
  std::unordered_map<std::pair<uint64_t, uint64_t>, double, KeyHash> acc;
  acc.reserve(1 << 20);
  const size_t N = n;
  for (int s = 0; s < 2; ++s)
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        const double v = h1e[p * N + q];
        if (v == 0.0) continue;
        const int modes[2] = {2 * p + s, 2 * q + s};
        const bool dag[2] = {true, false};
        add_product(acc, v, modes, dag, 2);
      }
  // 1/2 sum (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
  for (int s = 0; s < 2; ++s)
    for (int t = 0; t < 2; ++t)
      for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
          for (int r = 0; r < n; ++r)
            for (int u = 0; u < n; ++u) {
              const double v = eri[((p * N + q) * N + r) * N + u];
              const int P = 2 * p + s, R = 2 * r + t, U = 2 * u + t, Q = 2 * q + s;
              if (v == 0.0 || P == R || U == Q) continue;   // a+_P a+_P = a_Q a_Q = 0
              const int modes[4] = {P, R, U, Q};
              const bool dag[4] = {true, true, false, false};
              add_product(acc, 0.5 * v, modes, dag, 4);
            }
  // drop what cancelled (exactly or to rounding), group by flip mask, identity first
  double cmax = 0.0;
  for (const auto& kv : acc) cmax = std::max(cmax, std::fabs(kv.second));
  std::vector<std::pair<std::pair<uint64_t, uint64_t>, double>> terms;
  terms.reserve(acc.size());
  for (const auto& kv : acc)
    if (std::fabs(kv.second) > 1e-13 * cmax) terms.push_back(kv);
  std::sort(terms.begin(), terms.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  std::vector<uint64_t> mask, zs;
  std::vector<uint32_t> off;
  std::vector<double> coef;
  mask.push_back(0);
  off.push_back(0);
  for (const auto& t : terms) {
    if (t.first.first != mask.back()) {
      off.push_back((uint32_t)zs.size());
      mask.push_back(t.first.first);
    }
    zs.push_back(t.first.second);
    coef.push_back(t.second);
  }
  off.push_back((uint32_t)zs.size());
  if (zs.empty()) {   // keep the device arrays non-empty
    zs.push_back(0);
    coef.push_back(0.0);
  }
  hipFree(h->d_pl_mask); hipFree(h->d_pl_off); hipFree(h->d_pl_z); hipFree(h->d_pl_coef);
  h->d_pl_mask = nullptr; h->d_pl_off = nullptr; h->d_pl_z = nullptr; h->d_pl_coef = nullptr;
  h->pl_len = h->pl_strings = 0;
  if (hipMalloc(&h->d_pl_mask, mask.size() * 8) != hipSuccess || hipMalloc(&h->d_pl_off, off.size() * 4) != hipSuccess ||
      hipMalloc(&h->d_pl_z, zs.size() * 8) != hipSuccess || hipMalloc(&h->d_pl_coef, coef.size() * 8) != hipSuccess)
    return fail(ELOCAL_E_NOMEM, "device allocation failed in elocal_pauli_build");
  hipError_t e = hipMemcpy(h->d_pl_mask, mask.data(), mask.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_pl_off, off.data(), off.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_pl_z, zs.data(), zs.size() * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->d_pl_coef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "elocal_pauli_build copy");
  h->pl_len = (int64_t)mask.size();
  h->pl_strings = (int64_t)terms.size();
  return ELOCAL_OK;
}

int64_t elocal_pauli_count(elocal_t h, int what) {
  if (!h) return -1;
  return what == 0 ? h->pl_strings : h->pl_len;
}

size_t elocal_pauli_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t B) {
  if (!h) { fail(ELOCAL_E_INVALID, "handle is null"); return 0; }
  if (h->pl_len <= 0) { fail(ELOCAL_E_CONFIG, "no Pauli strings: call elocal_pauli_build first"); return 0; }
  AnsatzGeom G;
  if (make_geom(h, a, G) != ELOCAL_OK) return 0;
  const EvalPlan p = plan_eval(h, G, B, h->pl_len);
  return carve_eval(h, G, p, B, nullptr).bytes;
}

elocal_status elocal_eval_pauli(elocal_t h, elocal_stream s, const elocal_ansatz* a, const uint64_t* x, int64_t B,
                                void* ws, size_t ws_bytes, double* eloc) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (h->pl_len <= 0) return fail(ELOCAL_E_CONFIG, "no Pauli strings: call elocal_pauli_build first");
  AnsatzGeom G;
  if (elocal_status e = make_geom(h, a, G)) return e;
  if (G.precision != ELOCAL_BF16) return fail(ELOCAL_E_UNSUPPORTED, "the Pauli route runs the BF16 modes only");
  if (B < 0) return fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B);
  if (B == 0) return ELOCAL_OK;
  if (!a->theta || !x || !ws || !eloc) return fail(ELOCAL_E_INVALID, "null pointer argument");
  const EvalPlan p = plan_eval(h, G, B, h->pl_len);
  const EvalWs need = carve_eval(h, G, p, B, nullptr);
  if (ws_bytes < need.bytes) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need.bytes);
  if (elocal_status st = check_device(h)) return st;
  const EvalWs w = carve_eval(h, G, p, B, ws);
  hipStream_t st = (hipStream_t)s;
  MadeDev M = G.md;
  M.wfrag = w.frag;
  M.bias = w.bias;
  HIP_TRY(launch_pack_bf16(M, G.T, (const uint16_t*)a->theta, w.frag, (float*)w.bias, st), "pack launch");
  HIP_TRY(launch_pauli_diag(x, B, h->d_pl_off, h->d_pl_z, h->d_pl_coef, w.ediag, st), "diagonal launch");
  RowsArgs R{};
  R.sys = h->sys; R.made = M; R.x = x; R.B = B; R.lpx = w.lpx; R.zphi = w.zphi; R.logpsi = nullptr;
  HIP_TRY(launch_rows_bf16(R, G.hmax, G.nterms, st), "sample pass launch");
  EvalArgs E{};
  E.sys = h->sys; E.made = M; E.x = x; E.B = B; E.ediag = w.ediag; E.F = w.F; E.lpx = w.lpx; E.zphi = w.zphi;
  E.partial = w.partial; E.n_items = p.n_items; E.ips = p.ips; E.tpi = p.tpi;
  set_lds_args(E, p, G.bbytes);
  E.pl_mask = h->d_pl_mask; E.pl_off = h->d_pl_off; E.pl_z = h->d_pl_z; E.pl_coef = h->d_pl_coef;
  E.pl_len = (uint32_t)h->pl_len;
  const bool timed = h->timing && p.n_items > 0;
  const int slot = (int)(h->ring_pos % elocal_ctx::kRing);
  if (timed) HIP_TRY(hipEventRecord(h->ev_start[slot], st), "timing event");
  HIP_TRY(launch_eval_pauli_bf16(E, G.hmax, G.nterms, p.ldsw, p.lds, p.grid, p.waves, st), "Pauli eval launch");
  if (timed) {
    HIP_TRY(hipEventRecord(h->ev_stop[slot], st), "timing event");
    h->ring_pos++;
    h->recorded++;
  }
  HIP_TRY(launch_reduce(w.ediag, w.partial, B, p.ips, eloc, st), "reduce launch");
  return ELOCAL_OK;
}

// ----------------------------------------------------------------------------- BAS sampler
namespace {

struct SampleWs {
  void* frag;
  void* bias;
  uint64_t* pre[2];
  int64_t* w[2];
  double* probs;
  int64_t* counts;
  int64_t* off;
  int64_t* btot;
  int64_t* ucount;   // [2] prefix counts of the current and the next step (device)
  int64_t* overflow;
  size_t bytes;
};

SampleWs carve_sample(const elocal_ctx* h, const AnsatzGeom& G, int64_t cap, void* ws) {
  Carve c(ws);
  SampleWs w{};
  const size_t C = (size_t)std::max<int64_t>(cap, 1), W = h->sys.W;
  w.frag = c.take<char>(G.wbytes);
  w.bias = c.take<char>(G.bbytes);
  for (int k = 0; k < 2; ++k) {
    w.pre[k] = c.take<uint64_t>(C * W);
    w.w[k] = c.take<int64_t>(C);
  }
  w.probs = c.take<double>(4 * C);
  w.counts = c.take<int64_t>(4 * C);
  w.off = c.take<int64_t>(C);
  w.btot = c.take<int64_t>((C + 1023) / 1024);
  w.ucount = c.take<int64_t>(2);
  w.overflow = c.take<int64_t>(1);
  w.bytes = c.off;
  return w;
}

}  // namespace

size_t elocal_sample_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t max_unique) {
  if (!h) { fail(ELOCAL_E_INVALID, "handle is null"); return 0; }
  AnsatzGeom G;
  if (make_geom(h, a, G) != ELOCAL_OK) return 0;
  return carve_sample(h, G, max_unique, nullptr).bytes;
}

elocal_status elocal_sample(elocal_t h, elocal_stream s, const elocal_ansatz* a, int64_t n_samples, uint64_t seed,
                            int64_t max_unique, void* ws, size_t ws_bytes, uint64_t* x_out, int64_t* counts_out,
                            int64_t* n_unique) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  AnsatzGeom G;
  if (elocal_status e = make_geom(h, a, G)) return e;
  if (G.precision != ELOCAL_FP64) return fail(ELOCAL_E_UNSUPPORTED, "the sampler evaluates the ansatz in FP64 only");
  if (n_samples < 1 || n_samples > (1ll << 53))
    return fail(ELOCAL_E_INVALID, "n_samples=%lld outside [1, 2^53]", (long long)n_samples);
  if (max_unique < 1 || max_unique > 0xFFFFFFFFll) return fail(ELOCAL_E_INVALID, "max_unique outside [1, 2^32 - 1]");
  if (!a->theta || !ws || !x_out || !counts_out || !n_unique) return fail(ELOCAL_E_INVALID, "null pointer argument");
  const SampleWs need = carve_sample(h, G, max_unique, nullptr);
  if (ws_bytes < need.bytes) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need.bytes);
  if (elocal_status st = check_device(h)) return st;
  const SampleWs w = carve_sample(h, G, max_unique, ws);
  hipStream_t st = (hipStream_t)s;
  MadeDev M = G.md;
  M.wfrag = w.frag;
  M.bias = w.bias;
  HIP_TRY(launch_pack_f64(M, G.T, (const double*)a->theta, w.frag, (double*)w.bias, st), "pack launch");
  HIP_TRY(launch_bas_root(w.pre[0], w.w[0], h->sys.W, n_samples, &w.ucount[0], w.overflow, st), "root launch");
  // every step's launch sizes follow max_unique, the prefix counts stay on the device; the
  // last step writes the leaves straight into the caller's buffers
  int cur = 0;
  const int n = h->sys.n;
  for (int k = 0; k < n; ++k) {
    const bool last = k + 1 == n;
    HIP_TRY(launch_bas_step(h->sys, M, G.hmax, w.pre[cur], w.w[cur], &w.ucount[cur], &w.ucount[1 - cur], w.overflow,
                            k, seed, w.probs, w.counts, w.off, w.btot, last ? x_out : w.pre[1 - cur],
                            last ? counts_out : w.w[1 - cur], max_unique, st),
            "sampling step launch");
    cur = 1 - cur;
  }
  int64_t hv[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(&hv[0], &w.ucount[cur], sizeof(int64_t), hipMemcpyDeviceToHost, st), "count copy");
  HIP_TRY(hipMemcpyAsync(&hv[1], w.overflow, sizeof(int64_t), hipMemcpyDeviceToHost, st), "count copy");
  HIP_TRY(hipStreamSynchronize(st), "sampling sync");
  if (hv[1]) return fail(ELOCAL_E_WORKSPACE, "more than max_unique=%lld distinct prefixes at some orbital",
                         (long long)max_unique);
  *n_unique = hv[0];
  return ELOCAL_OK;
}

// ----------------------------------------------------------------------------- deduplicated eval
namespace {

struct DedupWs {
  double* ediag;
  double* F;
  void* frag;
  void* bias;
  uint64_t* xp;
  double* hval;
  int8_t* sign;
  uint32_t* exc;
  uint64_t* keys;
  uint32_t* ids;
  uint64_t* unique;
  float* lpx;
  double* lpx64;
  double* zphi;
  double* logpsi_u;
  int64_t* counters;
  uint64_t nslots;
  size_t bytes;
};

DedupWs carve_dedup(const elocal_ctx* h, const AnsatzGeom& G, int64_t B, void* ws) {
  Carve c(ws);
  DedupWs w{};
  const size_t Bs = (size_t)std::max<int64_t>(B, 1), total = Bs * h->sys.C;
  const size_t nS = h->sys.nSa + h->sys.nSb;
  uint64_t ns = 1024;
  while (ns < 2 * total) ns <<= 1;
  w.nslots = ns;
  w.ediag = c.take<double>(Bs);
  w.F = c.take<double>(std::max<size_t>(Bs * nS, 1));
  w.frag = c.take<char>(G.wbytes);
  w.bias = c.take<char>(G.bbytes);
  w.xp = c.take<uint64_t>(total);
  w.hval = c.take<double>(total);
  w.sign = c.take<int8_t>(total);
  w.exc = c.take<uint32_t>(total);
  w.keys = c.take<uint64_t>(ns);
  w.ids = c.take<uint32_t>(ns);
  w.unique = c.take<uint64_t>(total);
  if (G.precision == ELOCAL_BF16) w.lpx = c.take<float>(total * h->sys.n);
  else w.lpx64 = c.take<double>(total * h->sys.n);
  w.zphi = c.take<double>(total);
  w.logpsi_u = c.take<double>(2 * total);
  w.counters = c.take<int64_t>(2);
  w.bytes = c.off;
  return w;
}

}  // namespace

size_t elocal_dedup_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t B) {
  if (!h) { fail(ELOCAL_E_INVALID, "handle is null"); return 0; }
  AnsatzGeom G;
  if (make_geom(h, a, G) != ELOCAL_OK) return 0;
  return carve_dedup(h, G, B, nullptr).bytes;
}

elocal_status elocal_eval_dedup(elocal_t h, elocal_stream s, const elocal_ansatz* a, const uint64_t* x, int64_t B,
                                void* ws, size_t ws_bytes, double* eloc, double* logpsi, int64_t* n_distinct) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (h->sys.W != 1) return fail(ELOCAL_E_UNSUPPORTED, "deduplication needs one word per determinant (n <= 32)");
  AnsatzGeom G;
  if (elocal_status e = make_geom(h, a, G)) return e;
  if (B < 0) return fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B);
  if (B == 0) return ELOCAL_OK;
  if (!a->theta || !x || !ws || !eloc) return fail(ELOCAL_E_INVALID, "null pointer argument");
  if ((uint64_t)B * h->sys.C > 0xFFFFFFFFull) return fail(ELOCAL_E_UNSUPPORTED, "B x C exceeds 2^32 list entries");
  const DedupWs need = carve_dedup(h, G, B, nullptr);
  if (ws_bytes < need.bytes) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need.bytes);
  if (elocal_status st = check_device(h)) return st;
  const DedupWs w = carve_dedup(h, G, B, ws);
  hipStream_t st = (hipStream_t)s;
  const int64_t total = B * (int64_t)h->sys.C;
  MadeDev M = G.md;
  M.wfrag = w.frag;
  M.bias = w.bias;
  if (G.precision == ELOCAL_BF16)
    HIP_TRY(launch_pack_bf16(M, G.T, (const uint16_t*)a->theta, w.frag, (float*)w.bias, st), "pack launch");
  else
    HIP_TRY(launch_pack_f64(M, G.T, (const double*)a->theta, w.frag, (double*)w.bias, st), "pack launch");
  HIP_TRY(launch_prep(h->sys, x, B, w.ediag, w.F, st), "prep launch");
  HIP_TRY(launch_connect(h->sys, x, B, w.ediag, w.F, w.xp, w.hval, w.sign, w.exc, st), "connect launch");
  HIP_TRY(launch_dd_clear(w.keys, w.nslots, w.counters, st), "table clear launch");
  HIP_TRY(launch_dd_insert(w.xp, total, w.keys, w.nslots - 1, w.counters, st), "table insert launch");
  HIP_TRY(launch_dd_compact(w.keys, w.nslots, w.ids, w.unique, w.counters, st), "compaction launch");
  RowsArgs R{};
  R.sys = h->sys; R.made = M; R.x = w.unique; R.B = total; R.lpx = w.lpx; R.lpx64 = w.lpx64; R.zphi = w.zphi;
  R.logpsi = w.logpsi_u; R.count = w.counters;
  if (G.precision == ELOCAL_BF16) HIP_TRY(launch_rows_bf16(R, G.hmax, G.nterms, st), "distinct rows launch");
  else HIP_TRY(launch_rows_f64(R, G.hmax, st), "distinct rows launch");
  HIP_TRY(launch_dd_assemble(w.xp, w.hval, B, h->sys.C, w.keys, w.ids, w.nslots - 1, w.logpsi_u, eloc, logpsi,
                             w.counters, st), "assemble launch");
  if (n_distinct)
    HIP_TRY(hipMemcpyAsync(n_distinct, w.counters, sizeof(int64_t), hipMemcpyDeviceToDevice, st), "count copy");
  return ELOCAL_OK;
}

// ----------------------------------------------------------------------------- full sector / KPM
namespace {

struct SectorWs {
  double* partial;   // [waves][2]
  double* vec[3];    // recursion buffers (KPM only)
  size_t bytes;
  unsigned grid;
};

SectorWs carve_sector(const elocal_ctx* h, bool kpm, void* ws) {
  SectorWs w{};
  const int64_t dim = std::max<int64_t>(h->sector_dim, 1);
  w.grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((dim + 3) / 4, (int64_t)h->cu_count * 8));
  Carve c(ws);
  w.partial = c.take<double>((size_t)w.grid * 4 * 2);
  for (int k = 0; k < 3; ++k) w.vec[k] = kpm ? c.take<double>((size_t)dim) : nullptr;
  w.bytes = c.off;
  return w;
}

elocal_status check_sector(const elocal_ctx* h) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (h->sector_dim < 0)
    return fail(ELOCAL_E_UNSUPPORTED, "sector dimension of (%d, %d, %d) exceeds 2^31 - 1", h->sys.n, h->sys.na,
                h->sys.nb);
  return ELOCAL_OK;
}

}  // namespace

int64_t elocal_sector_dim(elocal_t h) { return h ? h->sector_dim : -1; }

size_t elocal_sector_workspace_bytes(elocal_t h, int kpm) {
  if (check_sector(h)) return 0;
  return carve_sector(h, kpm != 0, nullptr).bytes;
}

elocal_status elocal_sector_basis(elocal_t h, elocal_stream s, uint64_t* x) {
  if (elocal_status e = check_sector(h)) return e;
  if (!x) return fail(ELOCAL_E_INVALID, "x is null");
  if (elocal_status st = check_device(h)) return st;
  HIP_TRY(launch_sector_basis(h->sys, h->d_binom, h->sector_dim, h->sector_nb, x, (hipStream_t)s), "basis launch");
  return ELOCAL_OK;
}

elocal_status elocal_sector_apply(elocal_t h, elocal_stream s, double ch, const double* v, double cv, const double* z,
                                  double cz, double* y, void* ws, size_t ws_bytes, double* dots) {
  if (elocal_status e = check_sector(h)) return e;
  if (!v || !y || !ws) return fail(ELOCAL_E_INVALID, "null pointer argument");
  if (y == v || (z && y == z)) return fail(ELOCAL_E_INVALID, "y must not alias v or z");
  const SectorWs need = carve_sector(h, false, nullptr);
  if (ws_bytes < need.bytes) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need.bytes);
  if (elocal_status st = check_device(h)) return st;
  const SectorWs w = carve_sector(h, false, ws);
  hipStream_t st = (hipStream_t)s;
  HIP_TRY(launch_sector_apply(h->sys, h->d_binom, h->sector_dim, h->sector_nb, ch, cv, v, cz, z, y, w.partial, w.grid,
                              st), "sector apply launch");
  if (dots) HIP_TRY(launch_sector_dots(w.partial, (int64_t)w.grid * 4, dots, nullptr, -1, 0, st), "dots launch");
  return ELOCAL_OK;
}

elocal_status elocal_kpm_moments(elocal_t h, elocal_stream s, const double* alpha, int64_t n_moments, double a,
                                 double b, void* ws, size_t ws_bytes, double* moments) {
  if (elocal_status e = check_sector(h)) return e;
  if (!alpha || !ws || !moments) return fail(ELOCAL_E_INVALID, "null pointer argument");
  if (n_moments < 1) return fail(ELOCAL_E_INVALID, "n_moments=%lld < 1", (long long)n_moments);
  if (!(a > 0.0)) return fail(ELOCAL_E_INVALID, "scale a=%g must be positive", a);
  const SectorWs need = carve_sector(h, true, nullptr);
  if (ws_bytes < need.bytes) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need.bytes);
  if (elocal_status st = check_device(h)) return st;
  const SectorWs w = carve_sector(h, true, ws);
  hipStream_t st = (hipStream_t)s;
  const int64_t dim = h->sector_dim, nw = (int64_t)w.grid * 4;
  HIP_TRY(launch_norm2(alpha, dim, moments, st), "norm launch");   // Omega_0
  // a_1 = (H - b) a_0 / a; then a_{n+1} = 2 (H - b) a_n / a - a_{n-1}
  const double* prev = nullptr;
  const double* cur = alpha;
  int slot = 0;
  for (int64_t n = 0; 2 * n + 1 < n_moments; ++n) {
    double* nxt = w.vec[slot];
    const double ch = (n == 0 ? 1.0 : 2.0) / a, cv = -(n == 0 ? 1.0 : 2.0) * b / a;
    HIP_TRY(launch_sector_apply(h->sys, h->d_binom, dim, h->sector_nb, ch, cv, cur, -1.0, prev, nxt, w.partial,
                                w.grid, st), "sector apply launch");
    HIP_TRY(launch_sector_dots(w.partial, nw, nullptr, moments, n, n_moments, st), "moments launch");
    prev = cur;
    cur = nxt;
    slot = (slot + 1) % 3;
  }
  return ELOCAL_OK;
}

elocal_status elocal_kpm_line_shape(elocal_stream s, const double* moments, int64_t n_moments, const double* w,
                                    int64_t n_points, double* rho) {
  if (!moments || !w || !rho) return fail(ELOCAL_E_INVALID, "null pointer argument");
  if (n_moments < 1 || n_points < 0) return fail(ELOCAL_E_INVALID, "n_moments < 1 or n_points < 0");
  HIP_TRY(launch_line_shape(moments, n_moments, w, n_points, rho, (hipStream_t)s), "line shape launch");
  return ELOCAL_OK;
}

elocal_status elocal_stats(elocal_stream s, const double* eloc, const double* w, int64_t B, double* stats) {
  if (B < 1) return fail(ELOCAL_E_INVALID, "B=%lld < 1", (long long)B);
  if (!eloc || !w || !stats) return fail(ELOCAL_E_INVALID, "null pointer argument");
  HIP_TRY(launch_stats(eloc, w, B, stats, (hipStream_t)s), "stats launch");
  return ELOCAL_OK;
}

elocal_status elocal_grad(elocal_t h, elocal_stream s, const elocal_ansatz* a, const uint64_t* x,
                          const double* w, const double* eloc, int64_t B, void* ws, size_t ws_bytes,
                          double* stats, double* dtheta) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  AnsatzGeom G;
  if (elocal_status e = make_geom(h, a, G)) return e;
  if (B < 1) return fail(ELOCAL_E_INVALID, "B=%lld < 1", (long long)B);
  if (!a->theta || !x || !w || !eloc || !ws || !stats || !dtheta)
    return fail(ELOCAL_E_INVALID, "null pointer argument");
  const size_t need = carve_grad(h, G, B, nullptr, nullptr);
  if (ws_bytes < need) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need);
  if (elocal_status st = check_device(h)) return st;
  GradPlan P;
  carve_grad(h, G, B, ws, &P);
  P.theta = a->theta; P.x = x; P.w = w; P.eloc = eloc; P.B = B; P.stats = stats; P.dtheta = dtheta;
  HIP_TRY(launch_grad(P, (hipStream_t)s), "grad launch");
  return ELOCAL_OK;
}

elocal_status elocal_timing_enable(elocal_t h, int on) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (on && h->ev_start.empty()) {
    h->ev_start.resize(elocal_ctx::kRing);
    h->ev_stop.resize(elocal_ctx::kRing);
    for (int i = 0; i < elocal_ctx::kRing; ++i) {
      HIP_TRY(hipEventCreate(&h->ev_start[i]), "hipEventCreate");
      HIP_TRY(hipEventCreate(&h->ev_stop[i]), "hipEventCreate");
    }
  }
  h->timing = on != 0;
  return ELOCAL_OK;
}

elocal_status elocal_kernel_timing(elocal_t h, double* total_ms, int64_t* launches, int reset) {
  if (!h || !total_ms || !launches) return fail(ELOCAL_E_INVALID, "null pointer argument");
  const int64_t n = std::min<int64_t>(h->recorded, elocal_ctx::kRing);
  double tot = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const int slot = (int)((h->ring_pos - 1 - i + elocal_ctx::kRing * 4) % elocal_ctx::kRing);
    HIP_TRY(hipEventSynchronize(h->ev_stop[slot]), "hipEventSynchronize");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, h->ev_start[slot], h->ev_stop[slot]), "hipEventElapsedTime");
    tot += ms;
  }
  *total_ms = tot;
  *launches = n;
  if (reset) h->recorded = 0;
  return ELOCAL_OK;
}

elocal_status elocal_tune(elocal_t h, int param, int64_t value) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  switch (param) {
    case ELOCAL_TUNE_GRID: h->tune_grid = value; return ELOCAL_OK;
    case ELOCAL_TUNE_GROUPS: h->tune_groups = value; return ELOCAL_OK;
    case ELOCAL_TUNE_WAVES: h->tune_waves = value; return ELOCAL_OK;
    case ELOCAL_TUNE_COLS: h->tune_cols = value; return ELOCAL_OK;
  }
  return fail(ELOCAL_E_INVALID, "unknown tuning parameter %d", param);
}

int64_t elocal_launch_info(elocal_t h, const elocal_ansatz* a, int64_t B, int what) {
  if (!h) { fail(ELOCAL_E_INVALID, "handle is null"); return -1; }
  if (B < 0) { fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B); return -1; }
  AnsatzGeom G;
  if (make_geom(h, a, G) != ELOCAL_OK) return -1;
  const EvalPlan p = plan_eval(h, G, B);
  switch (what) {
    case ELOCAL_INFO_GRID: return p.grid;
    case ELOCAL_INFO_GROUPS: return p.tpi;
    case ELOCAL_INFO_WAVES: return p.waves;
    case ELOCAL_INFO_COLS: return p.cols;
    case ELOCAL_INFO_MAX_WAVES:
      return G.precision == ELOCAL_BF16 ? eval_waves_bf16(G.hmax, G.nterms, p.cols) : p.waves;
    case ELOCAL_INFO_ITEMS: return p.n_items;
    case ELOCAL_INFO_LDS_BYTES: return (int64_t)p.lds;
    case ELOCAL_INFO_INPLACE: return p.inplace ? 1 : 0;
  }
  fail(ELOCAL_E_INVALID, "unknown launch-info query %d", what);
  return -1;
}

elocal_status elocal_check_samples(elocal_t h, elocal_stream s, const uint64_t* x, int64_t B, void* ws,
                                   size_t ws_bytes, int64_t* n_bad) {
  if (!h) return fail(ELOCAL_E_INVALID, "handle is null");
  if (B < 0) return fail(ELOCAL_E_INVALID, "B=%lld is negative", (long long)B);
  if ((B > 0 && !x) || !ws) return fail(ELOCAL_E_INVALID, "null pointer argument");
  if (ws_bytes < 8) return fail(ELOCAL_E_WORKSPACE, "workspace %zu bytes < 8 needed", ws_bytes);
  if (elocal_status st = check_device(h)) return st;
  hipStream_t st = (hipStream_t)s;
  unsigned long long* bad = (unsigned long long*)ws;
  HIP_TRY(launch_check(h->sys, x, B, bad, st), "check launch");
  unsigned long long hbad = 0;
  HIP_TRY(hipMemcpyAsync(&hbad, bad, 8, hipMemcpyDeviceToHost, st), "check copy");
  HIP_TRY(hipStreamSynchronize(st), "check sync");
  if (n_bad) *n_bad = (int64_t)hbad;
  if (hbad) return fail(ELOCAL_E_CONFIG, "%llu sample(s) not in the (%d, %d) sector", hbad, h->sys.na, h->sys.nb);
  return ELOCAL_OK;
}

}  // extern "C"
