/*
 * elocal.h -- local energies of the second-quantised electronic Hamiltonian for an
 * autoregressive neural quantum state, on AMD Instinct MI355X (gfx950).
 *
 * What is computed (paper: "Scalable Neural Quantum State based Kernel Polynomial
 * Method for Optical Properties from the First Principle", arXiv 2506.07430):
 *
 *   E_loc(x) = sum_{x'} H_{x x'} Psi(x') / Psi(x)             (Results, local-energy
 *                                                               eq.; Algorithm 1)
 *   <E>      = sum_i w_i E_loc(x_i) / sum_i w_i               (Methods, batch estimator)
 *   G        = 2 Re sum_i wbar_i (E_loc(x_i) - <E>) d log Psi*(x_i)
 *                                                             (Methods, gradient
 *                                                               estimator, baseline <E>)
 *
 * for a batch of B unique occupation bitstrings x_i with multiplicities w_i. H is the
 * Hamiltonian of the Methods section built from one- and two-body integrals;
 * Psi = exp(A + i phi) is the masked autoregressive ansatz of the Results section.
 * The x' run over x and all its single and double excitations, enumerated in a fixed
 * canonical order (see elocal_connect).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Spin-orbitals: k = 2p + s for spatial orbital p (0-based) and spin s (0 = alpha/up,
 *   1 = beta/down) -- the paper's qubits 2i-1, 2i, made 0-based.
 * Bitstrings: W = ceil(2 n_orb / 64) little-endian uint64 words per determinant;
 *   spin-orbital k is bit (k % 64) of word (k / 64); unused high bits must be 0.
 * Signs: |x> = a+_{k1} a+_{k2} ... |vac> with k1 < k2 < ...; a_k and a+_k carry
 *   (-1)^(number of occupied spin-orbitals below k) (the Jordan--Wigner string).
 * Integrals: spatial, chemists' order, FP64, row-major:
 *   h1e[p*n + q] = h_pq, eri[((p*n + q)*n + r)*n + s] = (pq|rs), with
 *   H = sum_{pq,s} h_pq a+_{ps} a_{qs} + 1/2 sum_{pqrs,st} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}.
 *   eri must have the 8-fold permutational symmetry of real orbitals.
 * Ansatz parameters: one flat vector theta (layout at elocal_ansatz below).
 * Memory: every pointer argument of the compute calls is DEVICE memory owned by the
 *   caller; the library allocates nothing per call (all scratch lives in the
 *   caller's workspace). elocal_create copies the integrals (host pointers) to device
 *   memory owned by the handle.
 * Streams: compute calls only enqueue work on the given stream (NULL = the default
 *   stream) and return; they never synchronise, except elocal_check_samples and
 *   elocal_sample.
 * Errors: every call returns elocal_status; a non-zero status leaves the outputs
 *   unspecified and the handle usable. elocal_last_error() gives a message for the
 *   calling thread's last failure.
 * Threads: a handle is read-only after elocal_create (except for the timing and tuning
 *   calls at the end of this file); concurrent calls on one handle with separate
 *   workspaces and outputs are allowed.
 */
#ifndef ELOCAL_H
#define ELOCAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ELOCAL_OK = 0,
  ELOCAL_E_INVALID = 1,     /* bad argument: null pointer, size out of range, ...        */
  ELOCAL_E_CONFIG = 2,      /* a bitstring is not in the (n_alpha, n_beta) sector        */
  ELOCAL_E_WORKSPACE = 3,   /* workspace smaller than elocal_workspace_bytes()           */
  ELOCAL_E_NOMEM = 4,       /* device allocation in elocal_create failed                 */
  ELOCAL_E_DEVICE = 5,      /* HIP runtime error, or no gfx950 device is current         */
  ELOCAL_E_UNSUPPORTED = 6  /* shape outside what the kernels handle                     */
} elocal_status;

/* Arithmetic of the ansatz. H_{xx'}, ratios and every sum stay FP64 in every mode. */
enum {
  ELOCAL_FP64 = 0,   /* theta is double; ansatz on FP64 matrix cores                     */
  ELOCAL_BF16 = 1,   /* theta is bfloat16 (uint16 bit patterns); the ansatz products run
                        on the 16-bit matrix cores with FP32 accumulation: the weights are
                        used as fp16 (every bfloat16 value in [2^-17, 65504] is an fp16
                        number; smaller ones move by at most 2^-25), and each hidden
                        activation is carried as a hi+lo pair of fp16 values (<= 2^-22
                        relative, 2^-25 absolute for the smallest). Weights and hidden
                        activations must stay below 65504 in magnitude (fp16 range):
                        larger ones make the results non-finite. Measured against the FP64
                        oracle on the same parameters: a few 1e-7 Ha per local energy at
                        24 orbitals, ~1e-6 Ha at 60 orbitals (1.1e6 connected determinants) */
  ELOCAL_BF16X3 = 2  /* as ELOCAL_BF16 with three fp16 terms per activation (1.5x the
                        matrix-core work after the first layer; the FP32 accumulation then
                        dominates the error, so it is no more accurate in practice)        */
};

/* Operations, for elocal_workspace_bytes. */
enum { ELOCAL_OP_CONNECT = 0, ELOCAL_OP_EVAL = 1, ELOCAL_OP_GRAD = 2 };

typedef struct elocal_ctx* elocal_t;
typedef void* elocal_stream;   /* a hipStream_t */

/*
 * Ansatz description (host struct; theta itself is device memory).
 *
 * The network (Results, wavefunction ansatz; Fig. 1b): inputs are the 2n occupation
 * bits as 0/1; n_hidden >= 1 masked dense layers with ReLU; an output layer of 4n
 * logits ordered [orbital p][state s], s = x_{2p} + 2 x_{2p+1}; a phase head
 * phi = 2 pi sigmoid(w_phi . h_last + b_phi). Degrees: input bit k has degree
 * k/2 + 1; hidden unit j has degree (j mod (n-1)) + 1; a weight is used only if
 * input->hidden m >= d, hidden->hidden m' >= m, hidden->output(orbital p) p + 1 > m;
 * weights outside this mask are ignored (read as 0) and get gradient exactly 0.
 * Orbital p's 4 logits are restricted to the occupations that keep both electron
 * counts reachable (Results, number-conserving conditionals) and renormalised by a
 * softmax; A(x) = 1/2 sum_p log p_p(s_p).
 *
 * Flat layout of theta (P entries, P = elocal_num_params): for l = 0..n_hidden (the
 * last is the output layer) W_l[out_l][in_l] row-major then b_l[out_l], with
 * in_0 = 2n, out_l = widths[l] (l < n_hidden), out_{n_hidden} = 4n; then
 * w_phi[widths[n_hidden-1]], then b_phi[1].
 * Supported: 2 <= n <= 64, 1 <= n_hidden <= 8, every width a multiple of 32 in
 * [32, 256].
 */
typedef struct {
  int n_hidden;
  const int* widths;   /* host array [n_hidden]                                  */
  int precision;       /* ELOCAL_FP64 (theta: double), ELOCAL_BF16 or ELOCAL_BF16X3 (uint16) */
  const void* theta;   /* device pointer, P entries                              */
} elocal_ansatz;

/* Create a handle for one Hamiltonian and electron count (synchronous).
 * h1e [n*n], eri [n^4]: HOST pointers, copied. n_orb in [2, 64]; 0 <= n_alpha,
 * n_beta <= n_orb. Fails with ELOCAL_E_DEVICE when no gfx950 device is current. */
elocal_status elocal_create(const double* h1e, const double* eri, int n_orb, int n_alpha,
                            int n_beta, elocal_t* out);
elocal_status elocal_destroy(elocal_t h);

/* Number of connected determinants per sample, diagonal included (closed form):
 * C = 1 + sum_s n_s v_s + sum_s C(n_s,2) C(v_s,2) + n_a v_a n_b v_b, v_s = n - n_s.
 * Returns -1 for a null handle. No device work. */
int64_t elocal_num_connected(elocal_t h);
/* Words per bitstring, W = ceil(2n/64). */
int elocal_words(elocal_t h);
/* Length P of theta for n_orb and the hidden widths; -1 if unsupported. */
int64_t elocal_num_params(int n_orb, int n_hidden, const int* widths);

/* Bytes of device workspace a call needs (op = ELOCAL_OP_*; `a` may be NULL for
 * ELOCAL_OP_CONNECT). 0 on invalid arguments (elocal_last_error says why). */
size_t elocal_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t B, int op);

/*
 * Materialised connected lists (Results: the coupled configurations x^p of Algorithm 1,
 * here enumerated as fermionic excitations of x instead of Pauli flips).
 * x [B][W] in; out, for t in [0, C), in canonical order:
 *   xp   [B][C][W]  the determinant x'_t;
 *   hval [B][C]     H_{x'_t x} (FP64; sign included);
 *   sign [B][C]     <x'_t| a+_a a+_b a_j a_i |x> (+1/-1; +1 for the diagonal);
 *   exc  [B][C]     spin-orbitals i | j<<8 | a<<16 | b<<24, 0xFF for unused slots.
 * Order: t=0 the diagonal; alpha singles (i over occupied alpha ascending, outer;
 * a over virtual alpha ascending); beta singles; alpha-alpha doubles (occupied pairs
 * i<j lexicographic, outer x virtual pairs a<b lexicographic); beta-beta doubles;
 * alpha-beta doubles ((i,a) in alpha-single order, outer x (j,b) in beta-single
 * order). Values: diagonal sum_k h_kk + 1/2 sum_kl [(kk|ll) - (kl|lk)]; single
 * h_ai + sum_k [(ai|kk) - (ak|ki)]; double (ai|bj) - (aj|bi) (spin-orbital integrals).
 * Samples must be in the sector (unchecked here; see elocal_check_samples).
 * Outputs of any alignment are accepted. With xp and hval aligned to 16 bytes, exc to 8 and
 * sign to 2 (as fresh allocations are), and C >= 512, the lists are written two entries
 * per thread with vector stores, which is faster; the contents are the same.
 */
elocal_status elocal_connect(elocal_t h, elocal_stream s, const uint64_t* x, int64_t B,
                             void* ws, size_t ws_bytes, uint64_t* xp, double* hval,
                             int8_t* sign, uint32_t* exc);

/*
 * Local energies (Results, local-energy eq. and Algorithm 1; Methods, l_theta).
 * x [B][W] in; eloc [B][2] out (re, im); logpsi [B][2] out (A = log|Psi|, phi), may be
 * NULL. Every x' of the canonical list of every sample is generated, its matrix
 * element formed in FP64, the ansatz evaluated on it, and H_{xx'} exp(A'-A+i(phi'-phi))
 * summed in FP64 in a fixed order (bitwise repeatable).
 */
elocal_status elocal_eval(elocal_t h, elocal_stream s, const elocal_ansatz* a,
                          const uint64_t* x, int64_t B, void* ws, size_t ws_bytes,
                          double* eloc, double* logpsi);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): elocal_eval with the same arguments and
 * results, bit for bit, except that its scratch (what elocal_eval takes as ws) is a fixed
 * array of ELOCAL_NOALLOC_SCRATCH_MIB MiB in device memory, one per GPU, that the library
 * holds from the first elocal_create on that GPU until the process ends. The call allocates
 * nothing. Fails with ELOCAL_E_WORKSPACE when the batch needs more scratch than that
 * (elocal_workspace_bytes(h, a, B, ELOCAL_OP_EVAL) tells how much; e.g. 60 orbitals with
 * 1024 samples need about 52 MB). Every call on one GPU shares that GPU's array, and
 * nothing in it needs to start at zero: calls that overlap on one GPU (on different
 * streams, or from different threads) race and must be serialised by the caller.
 */
#define ELOCAL_NOALLOC_SCRATCH_MIB 64
elocal_status elocal_eval_noalloc(elocal_t h, elocal_stream s, const elocal_ansatz* a,
                                  const uint64_t* x, int64_t B, double* eloc, double* logpsi);

/*
 * Local energies of several systems in one persistent launch (Methods: the batch of a
 * training step split over independent summands; here systems of different size whose
 * connected lists differ in length by orders of magnitude).
 * n_sys in [1, ELOCAL_MAX_SYSTEMS]; hs, a, x, B, eloc, logpsi are HOST arrays of
 * n_sys entries (the pointers they hold are device memory, as in elocal_eval; logpsi
 * itself or any of its entries may be NULL). Every handle must belong to the current
 * device and every ansatz must have the same precision. System s gets exactly the
 * eloc[s] (and logpsi[s]) that elocal_eval(hs[s], ..., a[s], x[s], B[s]) gives: the
 * per-sample work and its summation order are the same; only the scheduling differs
 * (the fused kernel runs once over the work items of all systems, ordered by cost per
 * item, so no system leaves a tail of idle compute units behind it).
 * ws needs elocal_workspace_bytes_multi(...) bytes.
 */
enum { ELOCAL_MAX_SYSTEMS = 16 };
size_t elocal_workspace_bytes_multi(int n_sys, const elocal_t* hs, const elocal_ansatz* const* a,
                                    const int64_t* B);
elocal_status elocal_eval_multi(int n_sys, const elocal_t* hs, elocal_stream s,
                                const elocal_ansatz* const* a, const uint64_t* const* x,
                                const int64_t* B, void* ws, size_t ws_bytes, double* const* eloc,
                                double* const* logpsi);

/*
 * Batch autoregressive sampling (Results, parallel sampling: the BAS tree of unique
 * prefixes with multiplicities, pruned at every orbital, under the number-conserving
 * conditionals). Draws n_samples in [1, 2^53] determinants from |Psi|^2 and returns them as
 * *n_unique distinct determinants x_out [*n_unique][W] with counts counts_out [*n_unique]
 * (device buffers of max_unique entries, max_unique < 2^32), in tree order (prefix, then
 * state 0 = empty, 1 = alpha, 2 = beta, 3 = both). At orbital k every prefix i splits its
 * weight w by one multinomial draw, a chain of binomials over its reachable states in
 * ascending order: state s gets Binomial(w left, p_s / (p_s + later reachable p)), the last
 * reachable state the rest. A binomial with n p < 10 (p <= 1/2, else n minus the variate
 * for 1 - p) is drawn by inversion from 0, otherwise by BTRD (W. Hormann, J. Stat. Comput.
 * Simul. 46, 1993); attempt t of state s uses the two 53-bit uniforms of Philox4x32-10 at
 * counter (t, i, k, s), key (seed low, seed high): words (0,1) and (2,3), times 2^-53. The
 * ansatz is evaluated in FP64 (ELOCAL_FP64 only), so the tree is reproducible. The cost of
 * a step depends on the number of distinct prefixes only, not on n_samples. Synchronous
 * (once, at the end: the steps keep the prefix counts on the device); ELOCAL_E_WORKSPACE
 * if some orbital has more than max_unique distinct prefixes. Workspace:
 * elocal_sample_workspace_bytes.
 */
size_t elocal_sample_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t max_unique);
elocal_status elocal_sample(elocal_t h, elocal_stream s, const elocal_ansatz* a, int64_t n_samples,
                            uint64_t seed, int64_t max_unique, void* ws, size_t ws_bytes, uint64_t* x_out,
                            int64_t* counts_out, int64_t* n_unique);

/*
 * Local energies with every distinct connected determinant of the batch evaluated once
 * (the paper's deduplication of coupled configurations before the forward pass). The
 * lists are materialised (as elocal_connect), their determinants inserted into a hash
 * table, the ansatz run once per distinct determinant, and each E_loc assembled over
 * its list in canonical order. Same outputs as elocal_eval up to rounding (here A' - A
 * is a difference of totals). Worth it when the sector is small next to B x C (e.g. 8
 * orbitals: 369,664 list entries over at most 4,900 determinants); for large sectors
 * it only adds the materialisation. Needs n <= 32 and B x C < 2^32.
 * n_distinct (device, may be NULL) receives the number of distinct determinants.
 * Workspace: elocal_dedup_workspace_bytes (about 60 bytes per list entry).
 */
size_t elocal_dedup_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t B);
elocal_status elocal_eval_dedup(elocal_t h, elocal_stream s, const elocal_ansatz* a, const uint64_t* x,
                                int64_t B, void* ws, size_t ws_bytes, double* eloc, double* logpsi,
                                int64_t* n_distinct);

/*
 * The paper's own local-energy route (Results, local-energy equation over Pauli strings,
 * Algorithm 1 and the Pauli-element equation; Methods, Jordan--Wigner map): H is
 * rewritten as real-coefficient Pauli strings c X^m Z^z (on every qubit X before Z,
 * Y = i X Z; qubit k = spin-orbital k), grouped by flip mask m (the unique flips of
 * Algorithm 1, the identity first). E_loc(x) = sum over masks m of
 * H_m(x) Psi(x XOR m) / Psi(x), H_m(x) = sum over the mask's strings of
 * c (-1)^|z & (x XOR m)|; a flip that leaves the sector has Psi = 0 and contributes 0.
 * Every unique flip is run through the ansatz, as in the paper; elocal_eval runs only
 * the C connected determinants, with the same result.
 *
 * elocal_pauli_build: builds the strings from HOST integrals (the same h1e/eri as
 *   elocal_create; synchronous) and attaches them to the handle (replacing earlier ones).
 *   Needs 2 n <= 64. Coefficients below 1e-13 of the largest are dropped (cancellations).
 * elocal_pauli_count: what = 0 number of strings, 1 number of unique flip masks.
 * elocal_eval_pauli: E_loc [B][2] through the Pauli route (ELOCAL_BF16 / ELOCAL_BF16X3
 *   only); workspace elocal_pauli_workspace_bytes.
 */
elocal_status elocal_pauli_build(elocal_t h, const double* h1e, const double* eri);
int64_t elocal_pauli_count(elocal_t h, int what);
size_t elocal_pauli_workspace_bytes(elocal_t h, const elocal_ansatz* a, int64_t B);
elocal_status elocal_eval_pauli(elocal_t h, elocal_stream s, const elocal_ansatz* a, const uint64_t* x,
                                int64_t B, void* ws, size_t ws_bytes, double* eloc);

/*
 * Full-sector vectors and the kernel polynomial method (Methods, KPM for absorption
 * spectra; Results, KPM expansion of the dipole correlation function).
 *
 * A sector vector has one FP64 entry per determinant of the (n_alpha, n_beta) sector,
 * dim = C(n, n_alpha) C(n, n_beta) entries, at index r = rank_a * C(n, n_beta) + rank_b,
 * where the occupied spatial orbitals o_1 < ... < o_k of one spin have the
 * combinatorial-number-system rank sum_i C(o_i, i) (i = 1..k). All vectors are device
 * memory owned by the caller. H v is formed row by row from the same generator and
 * Slater--Condon values as elocal_eval (nothing per row is stored); every sum has a fixed
 * order, so results are bitwise repeatable.
 *
 * elocal_sector_dim: dim, or -1 when it exceeds 2^31 - 1 (the sector calls then fail with
 *   ELOCAL_E_UNSUPPORTED).
 * elocal_sector_workspace_bytes: workspace of elocal_sector_apply (kpm = 0) or of
 *   elocal_kpm_moments (kpm = 1: three recursion vectors are included).
 * elocal_sector_basis: x [dim][W], the determinant of every index.
 * elocal_sector_apply: y = ch (H v) + cv v + cz z (z may be NULL; y must not alias v or z);
 *   if dots is not NULL, dots[0] = <y|y> and dots[1] = <y|v> (device).
 *   The dipole vector |alpha> = mu |0> (mu = -sum_pq d_pq sum_s a+_ps a_qs - mu_c) is
 *   elocal_sector_apply on a handle created with h1e = -d and eri = 0, ch = 1, cv = -mu_c.
 * elocal_kpm_moments: Omega_0 .. Omega_{n_moments-1} of |alpha> for H~ = (H - b) / a
 *   (a > 0; the spectrum of H must lie inside (b - a, b + a)), by the recursion
 *   a_1 = H~ a_0, a_{n+1} = 2 H~ a_n - a_{n-1} and moment doubling
 *   Omega_{2n} = 2 <a_n|a_n> - Omega_0, Omega_{2n+1} = 2 <a_{n+1}|a_n> - Omega_1;
 *   moments [n_moments] is device memory; ceil(n_moments / 2) applications of H.
 * elocal_kpm_line_shape: rho(w~) = [g_0 Omega_0 + 2 sum_n g_n Omega_n T_n(w~)] /
 *   (pi sqrt(1 - w~^2)) at n_points points w~ in (-1, 1), with the Jackson kernel
 *   g_n = [(N - n + 1) cos(pi n / (N + 1)) + sin(pi n / (N + 1)) cot(pi / (N + 1))] / (N + 1),
 *   N = n_moments; rho approximates sum_k |<k|alpha>|^2 delta(w~ - E~_k).
 */
int64_t elocal_sector_dim(elocal_t h);
size_t elocal_sector_workspace_bytes(elocal_t h, int kpm);
elocal_status elocal_sector_basis(elocal_t h, elocal_stream s, uint64_t* x);
elocal_status elocal_sector_apply(elocal_t h, elocal_stream s, double ch, const double* v, double cv,
                                  const double* z, double cz, double* y, void* ws, size_t ws_bytes,
                                  double* dots);
elocal_status elocal_kpm_moments(elocal_t h, elocal_stream s, const double* alpha, int64_t n_moments,
                                 double a, double b, void* ws, size_t ws_bytes, double* moments);
elocal_status elocal_kpm_line_shape(elocal_stream s, const double* moments, int64_t n_moments,
                                    const double* w, int64_t n_points, double* rho);

/*
 * Energy statistics (Methods, batch estimator): stats[4] = (Re<E>, Im<E>,
 * sum_i w_i |E_i - <E>|^2 / sum_i w_i, sum_i w_i), from eloc [B][2] and w [B]
 * (device). B >= 1; sum w must be > 0. Fixed-order FP64 reduction.
 */
elocal_status elocal_stats(elocal_stream s, const double* eloc, const double* w, int64_t B,
                           double* stats);

/*
 * VMC gradient (Methods, gradient estimator with baseline b = <E>):
 *   dtheta = 2 sum_i wbar_i [Re(E_i - <E>) dA_i + Im(E_i - <E>) dphi_i],  wbar = w / sum w,
 * with <E> complex and held fixed; the ansatz forward at the B samples is recomputed
 * (nothing is kept from elocal_eval) and differentiated by hand in FP64. Inputs: x
 * [B][W], w [B], eloc [B][2] (from elocal_eval); outputs: stats [4] as elocal_stats,
 * dtheta [P] (double, theta's layout; masked weights get exactly 0).
 */
elocal_status elocal_grad(elocal_t h, elocal_stream s, const elocal_ansatz* a,
                          const uint64_t* x, const double* w, const double* eloc, int64_t B,
                          void* ws, size_t ws_bytes, double* stats, double* dtheta);

/*
 * Optional input check: counts samples of x [B][W] whose alpha/beta popcounts differ
 * from (n_alpha, n_beta) or whose unused high bits are set. Synchronises the stream.
 * Returns ELOCAL_E_CONFIG if any sample is bad (*n_bad, host, gets the count).
 * Needs a workspace of at least 8 bytes.
 */
elocal_status elocal_check_samples(elocal_t h, elocal_stream s, const uint64_t* x, int64_t B,
                                   void* ws, size_t ws_bytes, int64_t* n_bad);

/*
 * Timing of the dominant kernel (the fused local-energy kernel of elocal_eval; the
 * generator kernel of elocal_connect, without its per-sample preparation).
 * When enabled, each elocal_eval or elocal_connect on the handle (and each
 * elocal_eval_multi whose first handle it is) records a pair of HIP events around that
 * kernel on the caller's stream (a ring of 1024 pairs, reused in order).
 * elocal_kernel_timing waits for the recorded events, returns the summed milliseconds
 * and the number of launches recorded since the last reset (reset != 0 clears them).
 * These two calls mutate the handle: do not overlap them with other calls on it.
 */
elocal_status elocal_timing_enable(elocal_t h, int on);
elocal_status elocal_kernel_timing(elocal_t h, double* total_ms, int64_t* launches, int reset);

/*
 * Launch shape of the fused local-energy kernel (for the autotuner). A value <= 0
 * restores the built-in choice. elocal_eval_multi takes the grid, waves and tiles per pass
 * of its first handle (and each system's groups per item from its own handle).
 *   ELOCAL_TUNE_GRID:   blocks of the persistent grid-stride loop over work items.
 *   ELOCAL_TUNE_GROUPS: list-entry groups per work item (64 entries per group in BF16
 *                       mode, 16 in FP64 mode).
 *   ELOCAL_TUNE_WAVES:  waves per block of the BF16 kernels (at most what the kernel
 *                       variant is built for; ELOCAL_INFO_MAX_WAVES tells).
 *   ELOCAL_TUNE_COLS:   16-row tiles per network pass of the BF16 kernels: 1 or 2 (each
 *                       weight fragment then feeds twice the rows, in twice the registers,
 *                       so the variant is built for half the waves). Values no variant
 *                       provides for the ansatz (2 at width 256 in two-term mode, 1 in
 *                       three-term mode) fall back to the built-in choice.
 * Results do not depend on the launch shape except through the fixed per-item summation
 * order (rounding only). Mutates the handle: do not overlap with other calls on it.
 */
enum { ELOCAL_TUNE_GRID = 0, ELOCAL_TUNE_GROUPS = 1, ELOCAL_TUNE_WAVES = 2, ELOCAL_TUNE_COLS = 3 };
elocal_status elocal_tune(elocal_t h, int param, int64_t value);

/*
 * The launch shape elocal_eval would use for this handle, ansatz and batch size, after the
 * tuning above (host computation, no device work; -1 on invalid arguments):
 * ELOCAL_INFO_GRID blocks, ELOCAL_INFO_GROUPS groups per work item, ELOCAL_INFO_WAVES waves
 * per block, ELOCAL_INFO_COLS tiles per pass, ELOCAL_INFO_MAX_WAVES the waves per block the
 * kernel variant is built for, ELOCAL_INFO_ITEMS work items, ELOCAL_INFO_LDS_BYTES LDS per
 * block, ELOCAL_INFO_INPLACE 1 when the hidden layers are updated in place (one activation
 * array in registers; chosen when every hidden o-block pair j reads k-blocks j + 1 to j + 2
 * only), else 0.
 */
enum {
  ELOCAL_INFO_GRID = 0, ELOCAL_INFO_GROUPS = 1, ELOCAL_INFO_WAVES = 2, ELOCAL_INFO_COLS = 3,
  ELOCAL_INFO_MAX_WAVES = 4, ELOCAL_INFO_ITEMS = 5, ELOCAL_INFO_LDS_BYTES = 6, ELOCAL_INFO_INPLACE = 7
};
int64_t elocal_launch_info(elocal_t h, const elocal_ansatz* a, int64_t B, int what);

/* Message for the calling thread's last failure ("" if none). */
const char* elocal_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ELOCAL_H */
