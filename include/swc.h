/*
 * swc.h -- C ABI of the MI355X sparse wavefunction circuit (swc) library.
 *
 * The library simulates the factorized unitary coupled cluster circuit of
 * Mullinax & Tubman (arXiv:2301.05726) on one AMD Instinct MI355X (gfx950):
 *
 *   |Psi> = U_M ... U_2 U_1 |Psi_0>,   U_k = exp(theta_k (tau_k - tau_k^dag))
 *                                          (Results section, Eqs. 1-5)
 *
 * on a sparse state (determinant bitstring -> amplitude), discarding small
 * amplitudes after every factor (Methods section), and evaluates the energy
 * E = <Psi|H|Psi> / <Psi|Psi> of a second-quantized molecular Hamiltonian
 * and its exact gradient dE/dtheta by an adjoint (reverse) sweep.
 *
 * Conventions (fixed by this library; the paper states none):
 *  - spin-orbital q = 2p + s (p spatial orbital, s = 0 alpha, 1 beta);
 *    bit q of a determinant is set when q is occupied; n_qubits <= 64 (the
 *    paper's 32-spatial-orbital cap, Methods section);
 *  - |D> = a+_{q1} ... a+_{qN}|vac> with q1 < ... < qN (Jordan-Wigner order);
 *  - excitation row {i, j, a, b}: double tau = a+_a a+_b a_j a_i with i<j,
 *    a<b and {i,j}, {a,b} disjoint; single tau = a+_a a_i, encoded j=b=-1;
 *  - H = sum h_pq a+_{ps} a_{qs} + 1/2 sum (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}
 *    with real h1[p][q] (n x n, row major) and chemist-notation
 *    h2[p][q][r][s] (n^4, row major), n = n_qubits / 2, no nuclear term;
 *  - truncation: after every factor, every determinant with
 *    |amplitude| < threshold (strict, on the unit-norm state) is removed
 *    and the state is renormalised if anything was removed; threshold 0
 *    keeps everything (the circuit is then exactly unitary);
 *  - gradient: exact derivative with the truncation decisions of the
 *    forward sweep held fixed (equal to the true gradient at threshold 0).
 *
 * Precision: SWC_FP64 stores amplitudes in double; SWC_FP32 stores
 * amplitudes and the adjoint vector in float and rotates in float.  In both
 * modes the renormalisation, energy, sigma = H psi and gradient reductions
 * are done in double; all reductions are exact fixed-point sums, so every
 * result is bit-reproducible run to run.
 *
 * Memory and ownership: the caller allocates one device workspace of
 * swc_workspace_bytes(...) bytes (e.g. a torch tensor) and passes it to
 * swc_create; the library allocates no device memory itself, keeps that
 * pointer until swc_destroy, and never frees it.  Every other pointer is
 * used only during the call.  Pointers marked "device" must be device
 * memory of the current HIP device; "host" pointers are ordinary host
 * memory.  All device work is ordered on the stream given to swc_create;
 * calls return after their results are complete (they synchronize that
 * stream once at the end to read status flags).
 *
 * Errors: every int-returning call returns SWC_OK (0) or a negative code;
 * nothing throws across the ABI.  After SWC_ECAPACITY, SWC_EEMPTY or
 * SWC_EDEVICE the state held by the context is undefined until the next
 * swc_build_state; the context can always be destroyed.
 *
 * Environment (read by swc_create; results are bit-identical in every
 * setting): SWC_SWEEP=persistent runs each sweep as cooperative launches with
 * grid barriers instead of one launch per step; SWC_GRAPH=0 launches steps
 * directly instead of replaying captured graphs; SWC_FUSE=0 applies one
 * factor per launch at threshold 0; SWC_TABLE_MIN=n sets the smallest hash
 * index (default 2^18 slots); SWC_PROGRESS=1 waits after each range of steps
 * and reports it on stderr; SWC_KERNEL_TIMING=1 times every step launch (one
 * step per launch); SWC_GRID=n caps the sweep launches at about n blocks
 * (at least one per arena of entries; tuning); SWC_SPLIT=1 (0) always
 * (never) gives batch members one-factor step launches of their own, which
 * by default they get once their indexes reach 2^22 slots; SWC_HIOCC=1 (0)
 * always (never) runs the one-factor forward steps on their build for three
 * resident waves per SIMD, which by default they use from 2^22 index slots;
 * SWC_PFILTER=0 never probes through the index's presence filter, 1 always
 * where the library would (reverse steps at every index size, forward steps
 * from 2^22 slots), 2 always, forward steps at every size; by default a call
 * uses it unless the last forward sweep found the partner of more than one
 * rotated pair in four (never with entropy tracking, persistent sweeps or
 * the two-factor launches of threshold 0).
 */
#ifndef SWC_H
#define SWC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SWC_OK = 0,
  SWC_EINVAL = -1,    /* bad argument: sizes, indices, overlapping excitation
                         index sets, non-finite theta, threshold < 0, bad
                         determinant, workspace too small, batch index */
  SWC_ECAPACITY = -2, /* index, entry arenas or truncation log full */
  SWC_EEMPTY = -3,    /* truncation removed every determinant */
  SWC_EDEVICE = -4,   /* a HIP runtime error (text via swc_last_error) */
  SWC_ESTATE = -5     /* call order: no state built yet */
};

enum { SWC_FP64 = 0, SWC_FP32 = 1 };

typedef struct swc_ctx swc_ctx;

/* One UCC factor's excitation (Eq. 2): {i, j, a, b}, single: j = b = -1. */
typedef struct {
  int8_t i, j, a, b;
} swc_exc;

/* Counters of the last sweep(s), summed over the batch. */
typedef struct {
  int64_t n_live;        /* live determinants now (batch member 0) */
  int64_t det_updates;   /* sum over factors of live determinants visited (last forward sweep) */
  int64_t pair_updates;  /* rotated determinant pairs (last forward sweep) */
  int64_t inserts;       /* determinants created (last forward sweep) */
  int64_t pruned;        /* amplitudes removed by truncation (last forward sweep) */
  int64_t log_records;   /* truncation-log records of the last gradient sweep */
  int64_t table_slots;   /* current hash-index size per batch member (grows up to the capacity) */
  int64_t slots_used;    /* entries, alive and dead (= occupied index slots; batch member 0) */
  double fwd_ms;         /* device time of the last forward sweep */
  double energy_ms;      /* device time of the last energy evaluation */
  double rev_ms;         /* device time of the last reverse (adjoint) sweep */
  /* *_kernel_ms are filled only when the environment variable
     SWC_KERNEL_TIMING=1 was set at swc_create (an event pair is then
     recorded around every launch of these kernels, one factor per launch;
     the *_launches counts are then the timed launches): */
  double rotate_kernel_ms;   /* summed duration of the forward rotate kernels */
  int64_t rotate_launches;   /* rotate launches of the last forward sweep (one or two factors each;
                                one per batch member when members are launched apart) */
  double reverse_kernel_ms;  /* summed duration of the reverse kernels */
  int64_t reverse_launches;  /* reverse launches of the last adjoint sweep (likewise) */
  double sigma_kernel_ms;    /* duration of the sigma kernel (always filled) */
  int64_t partner_hits;      /* pairs whose partner existed (last forward sweep) */
  int64_t rehashes;          /* index growths during the last forward sweep */
  int64_t compactions;       /* rebuilds at its start that dropped the dead entries
                                of earlier sweeps (over 1/4 of the entries) */
  int64_t checkpoints;       /* snapshots taken by the last gradient sweep */
  int64_t sigma_partitions;  /* hash partitions of the two-electron-removed keys in the last pairing
                                sigma (0: hash probes were used) */
  int64_t shrinks;           /* always 0: the reverse sweep scans fewer entries as it goes
                                back without rebuilding anything */
  int64_t fwd_slots_scanned; /* entries (alive and dead) the last forward sweep's launches scanned */
  int64_t rev_slots_scanned; /* entries the reverse sweep scans to undo each factor, summed
                                over the factors (a two-factor launch scans its pair's once) */
  /* Totals over every swc_energy_and_grad call that completed since
     swc_create (a caller reads them before and after a series of calls
     instead of after each one): */
  int64_t grad_calls;           /* completed swc_energy_and_grad calls */
  double fwd_ms_total;          /* fwd_ms summed over those calls */
  double rev_ms_total;          /* rev_ms summed over those calls */
  double sigma_kernel_ms_total; /* sigma_kernel_ms summed over those calls */
  int64_t kernel_builds;        /* SWC_BUILD_* bits: the sweep kernel builds the last
                                   forward sweep and the reverse sweep after it launched */
} swc_stats;

/* Sweep kernel builds (swc_stats.kernel_builds). */
enum {
  SWC_BUILD_FWD = 1,          /* one factor per launch, forward */
  SWC_BUILD_FWD_ENT = 4,      /* the same, with the entropy sums */
  SWC_BUILD_FWD2 = 8,         /* two factors per launch (threshold 0), forward, home index slot preloaded */
  SWC_BUILD_FWD2_PRE = 16,    /* the same, four index slots per probe preloaded (one-pass states) */
  SWC_BUILD_REV = 32,         /* one factor per launch, reverse */
  SWC_BUILD_REV2 = 64,        /* two factors per launch, reverse, home slot preloaded */
  SWC_BUILD_REV2_PRE = 128,   /* the same, four index slots preloaded */
  SWC_BUILD_PERSISTENT = 256, /* persistent cooperative sweeps (SWC_SWEEP=persistent) */
  SWC_BUILD_FWD_HO = 512,     /* one factor per launch, forward, built for three resident waves per SIMD
                                 (indexes of 2^22 slots and more; SWC_HIOCC=1 always, 0 never) */
  SWC_BUILD_FWD_PF = 1024,    /* the one-factor forward launches probed through the presence filter */
  SWC_BUILD_REV_PF = 2048     /* the one-factor reverse launches probed through the presence filter */
};

/*
 * Bytes of device workspace needed for a context whose hash index may grow
 * to `capacity` slots per state (a power of two, >= 64; the determinants a
 * state holds, alive plus those removed during the current sweep, must stay
 * below 0.9 * capacity), `batch` independent states, circuits of up to
 * `max_factors` factors, and `log_capacity` truncation-log records per state
 * (0 selects capacity; a record, 20 bytes in FP32, saves the state of a
 * determinant removed earlier in the sweep that a later factor revives, for
 * the adjoint sweep).
 * The determinants of a state are dense arrays of entries (64 arenas with
 * room for 0.9 * capacity entries in all, so a state that outgrows the
 * capacity fails with SWC_ECAPACITY while its probes are still short); the
 * per-factor scans read the entries only.  The index maps a determinant to its entry; it starts small
 * after every reset to |Psi_0> and is rebuilt larger (x2 or more) during a
 * forward sweep when the entries near a growth limit (22.5% of its slots).
 * Beside the index lies its presence filter (one byte per index slot of
 * capacity): a partner lookup whose key the filter rules out reads no index
 * slot, which at the usual thresholds is nearly every lookup.
 * Returns 0 for invalid arguments.
 */
size_t swc_workspace_bytes(int n_qubits, uint64_t capacity, int prec, int batch, int64_t max_factors,
                           uint64_t log_capacity);

/*
 * Create a context.  n_alpha/n_beta electrons define the default reference
 * (Hartree-Fock determinant, bits 2p and 2p+1 occupied for p < n_alpha and
 * p < n_beta).  `workspace` (device, >= swc_workspace_bytes) stays owned by
 * the caller and must outlive the context; `stream` is a hipStream_t (NULL
 * for the default stream).  On success *out receives the context.
 */
int swc_create(swc_ctx** out, int n_qubits, int n_alpha, int n_beta, uint64_t capacity, int prec, int batch,
               int64_t max_factors, uint64_t log_capacity, void* workspace, size_t ws_bytes, void* stream);

/*
 * Set the initial state |Psi_0> (Eq. 1) of every batch member: `n` host
 * determinants and amplitudes (host arrays; duplicates or bits at or above
 * n_qubits -> SWC_EINVAL).  The state is normalised.  n = 0 selects the
 * Hartree-Fock reference.  Resets the current state to |Psi_0>.
 */
int swc_build_state(swc_ctx* ctx, const uint64_t* dets, const double* amps, int64_t n);

/*
 * Apply U_M ... U_1 (Eq. 3; factor k in the closed form of Eqs. 4-5) to the
 * current state of every batch member, truncating after each factor.
 * theta: device double [batch][M]; exc: host swc_exc[M]; 0 <= M <= max_factors.
 */
int swc_apply_ucc(swc_ctx* ctx, const double* theta, const swc_exc* exc, int64_t M, double threshold);

/*
 * E[b] = <psi_b|H|psi_b> / <psi_b|psi_b> of the current states: the
 * energy objective the paper evaluates on the final state of the circuit
 * (Results section), as a Rayleigh quotient of the second-quantized H above.
 * h1: device double [n][n]; h2: device double [n][n][n][n]; E: device double [batch].
 */
int swc_energy(swc_ctx* ctx, const double* h1, const double* h2, double* E);

/*
 * E(theta) and dE/dtheta for every batch member, starting from |Psi_0>
 * (forward sweep with truncation, energy, adjoint sweep).  The paper does not
 * say how its optimizer (SLSQP, Methods section) obtains gradients; this is
 * the exact derivative of E with the truncation decisions of the forward
 * sweep held fixed (the limit of central differences whenever no amplitude
 * crosses the cut; the true gradient at threshold 0), computed by running the
 * factors backwards on the state and on lambda = P (H - E) psi.  Arguments as
 * in swc_apply_ucc and swc_energy; grad: device double [batch][M].  On return
 * the current state is |Psi_0> again.
 */
int swc_energy_and_grad(swc_ctx* ctx, const double* theta, const swc_exc* exc, int64_t M, double threshold,
                        const double* h1, const double* h2, double* E, double* grad);

/*
 * Checkpoints of the gradient sweep.  The adjoint sweep rebuilds each
 * forward state psi_{k-1} from psi_k by inverting step k exactly (the support
 * is rebuilt bit for bit from per-entry step tags and the truncation log);
 * in floating point the rebuilt amplitudes drift by rounding, step after
 * step.  With checkpoints on, swc_energy_and_grad snapshots the live
 * (determinant, amplitude) pairs after forward steps interval, 2*interval,
 * ... (< M), and the adjoint sweep writes each snapshot back over the state
 * it has rebuilt for the same step, so the drift never spans more than
 * `interval` steps.  The results match the uncheckpointed sweep within
 * rounding; the FP32 gradient of a long circuit is closer to the FP64 one.
 *
 * swc_checkpoint_bytes: size of the device buffer for circuits of up to
 * max_factors factors, snapshots of up to max_entries live determinants per
 * batch member (12 bytes per entry in FP32, 16 in FP64), or 0 for invalid
 * arguments.  swc_set_checkpoints: `buffer` (device, 256-byte aligned, owned
 * by the caller, kept until the next call or swc_destroy) turns checkpoints
 * on; interval <= 0 turns them off (buffer may be NULL).  A snapshot with
 * more live determinants than max_entries makes swc_energy_and_grad return
 * SWC_ECAPACITY.
 */
size_t swc_checkpoint_bytes(int prec, int batch, int64_t max_factors, int64_t interval, uint64_t max_entries);
int swc_set_checkpoints(swc_ctx* ctx, int64_t interval, uint64_t max_entries, void* buffer, size_t bytes);

/*
 * Wavefunction entropy along the circuit (Eq. 6: S = -sum_I |c_I|^2 ln |c_I|^2
 * over the normalised state).  swc_track_entropy(ctx, 1) makes every later
 * forward sweep (swc_apply_ucc, swc_energy_and_grad) record S of the state it
 * starts from and after each of its M factors (after truncation); the sums are
 * exact fixed-point reductions, so S is bit-reproducible.  While on, factors
 * are applied one per launch.  swc_get_entropy copies those M + 1 values of
 * batch member b into the host array S (n >= M + 1); SWC_ESTATE if the last
 * forward sweep did not track it.
 */
int swc_track_entropy(swc_ctx* ctx, int on);

/*
 * N_MAX / N_CUT truncation (Methods section): after the threshold cut of every
 * factor of later forward sweeps, when more than n_max determinants are live,
 * keep the n_cut of largest |c| (ties: the smaller determinant bit pattern) and
 * remove the rest like a threshold cut (renormalisation, exact adjoint).  The
 * n_cut-th |c| is found by a radix selection on the device after every
 * factor (several small launches per factor while on).  n_max = n_cut = 0
 * turns it off; otherwise 1 <= n_cut <= n_max, else SWC_EINVAL.
 */
int swc_set_topk(swc_ctx* ctx, uint64_t n_max, uint64_t n_cut);

/*
 * Scratch for sigma = H psi (energy; Results section) by pairing instead of
 * hash probes.  Two determinants differ by a double excitation exactly when
 * removing two electrons from each leaves the same pattern K, and by a single
 * one when removing one electron from each does: every live determinant
 * emits one record (K, index) per pair of its occupied spin-orbitals, then
 * one per occupied spin-orbital; the records are radix-sorted by K on the
 * device, and each group sums <I|H|J> c_J over its members (exact
 * fixed-point sums).  Only connections present in the state are touched;
 * absent ones are never probed.  The diagonal keeps its own path.  `buffer` (device,
 * 256-byte aligned, caller-owned, kept until the next call or swc_destroy):
 * about 41 bytes per record plus 24 bytes per live determinant; records
 * beyond it are processed in hash partitions of K (pairing is skipped when
 * the buffer cannot hold the accumulators and 4096 records).  mode: 0 = pairing when the record
 * count (live determinants x pairs of electrons) reaches 2^22, 1 = always,
 * 2 = never (NULL buffer: never).  Results agree with the probing path to
 * rounding; both are bit-reproducible.
 */
int swc_set_sigma_scratch(swc_ctx* ctx, void* buffer, size_t bytes, int mode);
int swc_get_entropy(swc_ctx* ctx, int b, double* S, int64_t n);

/*
 * State size along the circuit.  swc_track_live(ctx, 1) makes every later
 * forward sweep (swc_apply_ucc, swc_energy_and_grad) count the live
 * determinants of each step (one more sharded atomic per wave and step; off
 * by default).  swc_get_live_counts: n[k] (k = 0..M-1) is the number of live
 * determinants of batch member b when step k+1 of the last forward sweep
 * began, after the truncation of step k; n[M] is the number after the last
 * step.  n is a host array of len >= M + 1; the sum of n[0..M-1] is the
 * sweep's det-updates.  SWC_ESTATE if the last forward sweep did not count.
 */
int swc_track_live(swc_ctx* ctx, int on);
int swc_get_live_counts(swc_ctx* ctx, int b, int64_t* n, int64_t len);

/*
 * Copy the current state of batch member b to host arrays sorted by
 * determinant (amplitudes normalised, in double).  *n_out receives the
 * number of determinants; SWC_ECAPACITY if it exceeds `cap` (nothing copied).
 */
int swc_get_state(swc_ctx* ctx, int b, uint64_t* dets, double* amps, int64_t cap, int64_t* n_out);

int swc_get_stats(swc_ctx* ctx, swc_stats* out);

/* Static text for an error code; swc_last_error gives the last HIP/argument message. */
const char* swc_strerror(int code);
const char* swc_last_error(void);

void swc_destroy(swc_ctx* ctx);

/*
 * For callers that cannot allocate device memory (code whose launches are
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc): the energy E = <Psi|H|Psi> / <Psi|Psi> of the state with the n
 * distinct determinants dets[i] and amplitudes amps[i] (device arrays, FP64),
 * the value swc_build_state + swc_energy give for it (FP64 amplitudes; equal up
 * to the rounding of the norm, which this call does not apply), without a
 * context and with no device allocation: the index, entries, compact arrays
 * and counters live in one static device array of SWC_NOALLOC_SCRATCH_BYTES
 * that every device the library runs on holds until the process ends.
 *   n_qubits  even, 2..64 (spin-orbital q = 2p + spin, as everywhere here)
 *   n         1..SWC_NOALLOC_MAX_DETS determinants; larger states: SWC_EINVAL
 *   h1, h2    device, n_qubits/2 spatial orbitals, as for swc_energy
 *   E         device, one double (written on the stream)
 *   stream    the HIP stream every kernel of the call runs on
 * The call waits for the stream at its end, to report what the device checks
 * found: SWC_EINVAL for a repeated determinant, a bit at or above n_qubits, a
 * non-finite amplitude or a zero norm (E is then meaningless).  Calls on one
 * device share its array, which keeps the last call's contents (the call
 * clears what it reads): calls that overlap on one device, from several host
 * threads or streams, race.
 */
#define SWC_NOALLOC_MAX_DETS 65536
#define SWC_NOALLOC_SCRATCH_BYTES 8133120 /* 7.8 MiB per device */
int swc_energy_noalloc(int n_qubits, const uint64_t* dets, const double* amps, int64_t n, const double* h1,
                       const double* h2, double* E, void* stream);

/*
 * Host-only helpers (no device work; usable on machines without a GPU).
 * swc_validate_excitations: SWC_OK or SWC_EINVAL for an excitation list.
 * swc_factor_masks: per factor k writes masks[3k..3k+2] =
 *   {occupied-side mask, virtual-side mask, sign mask}; a determinant D is
 *   the lower member of a pair when (D & occ) == occ and (D & vir) == 0,
 *   the upper member when the roles swap, and the fermionic sign of
 *   tau|lower> is (-1)^popcount(D & sign) for either member.
 */
int swc_validate_excitations(int n_qubits, const swc_exc* exc, int64_t M);
int swc_factor_masks(int n_qubits, const swc_exc* exc, int64_t M, uint64_t* masks);

#ifdef __cplusplus
}
#endif

#endif /* SWC_H */
