// Evaluate every distinct connected determinant of a batch once: an open-addressing
// hash table over the materialised lists (one 64-bit word per determinant), compaction
// of the distinct keys, and the per-sample assembly of E_loc from the ansatz values of
// the distinct determinants. Identifiers come from atomic counters, so they depend on
// scheduling; no result does (every sum runs over a sample's list in canonical order).
#include "elocal_internal.hpp"
#include "kernels.hpp"

namespace elocal {

constexpr uint64_t kEmptyKey = ~0ull;   // never a determinant: bits above 2n are zero (n <= 32)

__device__ __forceinline__ uint64_t mix64(uint64_t k) {
  // splitmix64 finaliser
  k ^= k >> 30;
  k *= 0xBF58476D1CE4E5B9ull;
  k ^= k >> 27;
  k *= 0x94D049BB133111EBull;
  k ^= k >> 31;
  return k;
}

__global__ void k_dd_clear(uint64_t* __restrict__ keys, uint64_t nslots, int64_t* __restrict__ counters) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nslots) keys[i] = kEmptyKey;
  if (i < 2) counters[i] = 0;
}

// Insert every x' (linear probing; the table has at least twice as many slots as keys,
// so a free slot or the key itself is always found within nslots probes; a probe count
// beyond that sets counters[1] and stops).
__global__ void k_dd_insert(const uint64_t* __restrict__ xp, int64_t total, uint64_t* __restrict__ keys,
                            uint64_t mask, int64_t* __restrict__ counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint64_t key = xp[i];
  uint64_t h = mix64(key) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&keys[h], (unsigned long long)kEmptyKey, (unsigned long long)key);
    if (prev == kEmptyKey || prev == key) return;
    h = (h + 1) & mask;
  }
  atomicAdd((unsigned long long*)&counters[1], 1ull);
}

// Give every occupied slot an identifier and list its key.
__global__ void k_dd_compact(const uint64_t* __restrict__ keys, uint64_t nslots, uint32_t* __restrict__ ids,
                             uint64_t* __restrict__ unique, int64_t* __restrict__ counters) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nslots) return;
  const uint64_t key = keys[i];
  if (key == kEmptyKey) return;
  const unsigned long long id = atomicAdd((unsigned long long*)&counters[0], 1ull);
  ids[i] = (uint32_t)id;
  unique[id] = key;
}

__device__ __forceinline__ uint32_t dd_lookup(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ ids,
                                              uint64_t mask, uint64_t key) {
  uint64_t h = mix64(key) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const uint64_t k = keys[h];
    if (k == key) return ids[h];
    if (k == kEmptyKey) break;
    h = (h + 1) & mask;
  }
  return 0xFFFFFFFFu;
}

// E_loc of every sample: one wave per sample, lanes over its list in canonical order,
// ratio exp(A' - A + i (phi' - phi)) from the distinct determinants' log psi.
__global__ void __launch_bounds__(256) k_dd_assemble(const uint64_t* __restrict__ xp, const double* __restrict__ hval,
                                                     int64_t B, uint32_t C, const uint64_t* __restrict__ keys,
                                                     const uint32_t* __restrict__ ids, uint64_t mask,
                                                     const double* __restrict__ logpsi_u, double* __restrict__ eloc,
                                                     double* __restrict__ logpsi_out, int64_t* __restrict__ counters) {
  const int lane = threadIdx.x & 63;
  const int64_t b = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (b >= B) return;
  const uint64_t* xb = xp + (size_t)b * C;
  const uint32_t id0 = dd_lookup(keys, ids, mask, xb[0]);
  if (id0 == 0xFFFFFFFFu) {
    if (lane == 0) atomicAdd((unsigned long long*)&counters[1], 1ull);
    return;
  }
  const double A0 = logpsi_u[2 * id0], phi0 = logpsi_u[2 * id0 + 1];
  double re = 0.0, im = 0.0;
  for (uint32_t t = 1 + lane; t < C; t += 64) {
    const double hv = hval[(size_t)b * C + t];
    if (hv == 0.0) continue;
    const uint32_t id = dd_lookup(keys, ids, mask, xb[t]);
    if (id == 0xFFFFFFFFu) {
      atomicAdd((unsigned long long*)&counters[1], 1ull);
      continue;
    }
    double sn, cs;
    sincos(logpsi_u[2 * id + 1] - phi0, &sn, &cs);
    const double mag = hv * exp(logpsi_u[2 * id] - A0);
    re += mag * cs;
    im += mag * sn;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    re += __shfl_xor(re, off);
    im += __shfl_xor(im, off);
  }
  if (lane == 0) {
    eloc[2 * b] = hval[(size_t)b * C] + re;
    eloc[2 * b + 1] = im;
    if (logpsi_out) {
      logpsi_out[2 * b] = A0;
      logpsi_out[2 * b + 1] = phi0;
    }
  }
}

// ----------------------------------------------------------------------------- launchers
hipError_t launch_dd_clear(uint64_t* keys, uint64_t nslots, int64_t* counters, hipStream_t st) {
  const uint64_t n = nslots > 2 ? nslots : 2;
  hipLaunchKernelGGL(k_dd_clear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, keys, nslots, counters);
  return hipGetLastError();
}

hipError_t launch_dd_insert(const uint64_t* xp, int64_t total, uint64_t* keys, uint64_t mask, int64_t* counters,
                            hipStream_t st) {
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd_insert, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, xp, total, keys, mask,
                     counters);
  return hipGetLastError();
}

hipError_t launch_dd_compact(const uint64_t* keys, uint64_t nslots, uint32_t* ids, uint64_t* unique, int64_t* counters,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_dd_compact, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, st, keys, nslots, ids, unique,
                     counters);
  return hipGetLastError();
}

hipError_t launch_dd_assemble(const uint64_t* xp, const double* hval, int64_t B, uint32_t C, const uint64_t* keys,
                              const uint32_t* ids, uint64_t mask, const double* logpsi_u, double* eloc,
                              double* logpsi_out, int64_t* counters, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dd_assemble, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, st, xp, hval, B, C, keys, ids, mask,
                     logpsi_u, eloc, logpsi_out, counters);
  return hipGetLastError();
}

}  // namespace elocal
