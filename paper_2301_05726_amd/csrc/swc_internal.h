// Internal definitions shared by the kernels (swc_kernels.hip) and the host
// side of the C ABI (swc_api.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace swc {

// ---------------------------------------------------------------------------
// state layout: dense entry arrays + a hash index
// ---------------------------------------------------------------------------
// The determinants of a state are entries of dense arrays (Slot<T>, plus the
// AuxF side array for float states), split into NA arenas: a launch appends
// the entries it creates to the arena of the creating wave, so the entries of
// an arena are in creation order.  The sweeps scan the entries, never the
// empty slots of a hash table.  A separate open-addressed index (linear
// probing on a 64-bit mixer) maps a determinant to its entry.
//
// An entry's meta holds a state bit and a step tag (1-based factor index
// within the current sweep, 0 = before it):
//   alive:  meta = born tag          (step that created the entry)
//   dead:   meta = DEAD | death tag   (step whose truncation removed it)
// born keeps the creation tag of dead entries (needed when the reverse sweep
// resurrects them).  A dead entry keeps its key (it stays in the index) and,
// for a death during the current sweep, its pre-truncation amplitude.
constexpr uint64_t EMPTY_KEY = ~0ull;
constexpr uint64_t NO_LIMIT = ~0ull;  // index occupancy limit of an index that cannot grow
constexpr int SH = 64;  // shards of each per-step accumulator
constexpr uint32_t DEAD = 0x80000000u;
constexpr uint32_t TAG = 0x7fffffffu;
constexpr int NA = 64;                   // arenas per state
constexpr int ID_POS_BITS = 26;          // entry id = arena << 26 | position in the arena
constexpr uint32_t ID_POS_MASK = (1u << ID_POS_BITS) - 1u;
constexpr uint32_t NO_ID = ~0u;          // an index slot whose entry id is not written yet
constexpr uint32_t NB_UNSET = ~0u;       // no forward launch began at this step

// status flags (Counters::flags)
enum : uint32_t {
  F_TABLE_FULL = 1u,
  F_LOG_FULL = 2u,
  F_BAD_THETA = 4u,
  F_INCONSISTENT = 8u,
  F_TIMEOUT = 16u,  // a grid barrier of a persistent sweep gave up waiting
  F_BAD_INPUT = 32u,  // a device-side input list failed its check (k_check_list)
};

// grid-barrier state of the persistent sweeps (one 256-byte line)
struct alignas(256) Sync {
  unsigned int count;
  unsigned int timeout;
};

// 128-bit two's complement fixed point, value = (hi:lo) * 2^-96.  Every
// reduction of floating-point terms is done by converting each term to this
// format and adding integers, so sums are exact and order independent.
struct Fx {
  unsigned long long lo;
  unsigned long long hi;
};

// Accumulator of Fx terms updated by atomics that return nothing (a wave
// does not wait for them): the 128-bit term is split into 42-bit limbs
// (the top one signed), each summed in its own 64-bit word; a word takes at
// most 2^22 additions before the value is read back, so no limb overflows
// and the sum is exact.
struct Fx3 {
  unsigned long long l[3];
};

// Event counters are sharded: a block adds to shard (blockIdx.x % CSH), each
// shard in its own 128-byte line, so concurrent atomics rarely meet.
constexpr int CSH = 32;
enum : int {
  C_LIVE = 0,  // alive entries
  C_OCC,       // entries (alive + dead) = occupied index slots
  C_DU,        // det visits (forward)
  C_PAIRS,     // rotated pairs (forward)
  C_INS,       // created entries (forward)
  C_PRUNED,    // truncated amplitudes (forward)
  C_HITS,      // rotated pairs whose partner existed (forward)
  C_NCNT
};
// shard 0 only: entry positions scanned by the last forward / reverse sweep
constexpr int C_FSCAN = 14, C_RSCAN = 15;
struct alignas(128) CShard {
  unsigned long long v[16];
};

// Shards of the energy sums sum c sigma and sum c^2 (exact, 3 limbs each):
// a block of the energy reduction adds to shard (blockIdx.x % ESH) with
// non-returning atomics; the final kernel adds the shards.
constexpr int ESH = 16;
struct alignas(128) ESum {
  Fx3 num, den;
};

// per-state device counters
struct Counters {
  CShard sh[CSH];
  unsigned long long logcnt;    // truncation-log records this sweep
  unsigned long long ncompact;  // entries in the compact arrays
  unsigned int flags;
  unsigned int stop;            // (member 0 only) first forward step that must not run; ~0u = none
  double S;                     // current renormalisation scale: psi = S * raw
  Fx num;                       // sum c sigma
  Fx den;                       // sum c^2
  double E;
  double pad2;
  ESum es[ESH];
};

inline unsigned long long counter_total(const Counters& c, int which) {
  unsigned long long t = 0;
  for (int s = 0; s < CSH; ++s) t += c.sh[s].v[which];
  return t;
}

struct FacMask {
  uint64_t occ, vir, sgn;
};

struct Trig {
  double c, s, cm1;  // cos, sin, cos - 1 (= -2 sin^2(theta/2))
};

// Entries.  float states: 16-byte {key, amp, meta} plus an 8-byte side
// array {lam, born}; double states: one 32-byte entry.  lam is the adjoint
// amplitude of the reverse sweep, born the creation tag.
template <class T>
struct Slot;
template <>
struct alignas(16) Slot<float> {
  uint64_t key;
  float amp;
  uint32_t meta;
};
template <>
struct alignas(32) Slot<double> {
  uint64_t key;
  double amp;
  double lam;
  uint32_t meta;
  uint32_t born;
};
struct alignas(8) AuxF {
  float lam;
  uint32_t born;
};

// index slot: determinant and its entry id (EMPTY_KEY: free)
struct alignas(16) Idx {
  uint64_t key;
  uint32_t id;
  uint32_t pad;
};

// The state of every batch member: member b's entries at b*E (E = NA*A; arena
// s at s*A), its index slots at b*Hcap (H of them in use).
struct Tab {
  void* ent;     // Slot<T>[B*E]
  void* aux;     // AuxF[B*E] for float states, unused for double
  Idx* idx;      // Idx[B*Hcap]
  uint32_t* ac;  // entries per arena [B*NA] between sweeps (a sweep keeps its counts per step)
  uint64_t H;    // index slots in use per member (power of two)
  uint64_t Hcap; // index slots reserved per member
  uint64_t A;    // entries per arena (<= 2^ID_POS_BITS)
};

// Presence filter of an index (a blocked Bloom filter over the keys it
// holds): member b's words at w + b * stride, n = H/8 of them in use (one
// 64-bit word per 8 index slots).  w = nullptr: none.  Kept apart from Tab so
// that the step kernels without it take exactly the arguments they need.
struct Pf {
  uint64_t* w = nullptr;
  uint64_t n = 0;
  uint64_t stride = 0;
};

// truncation log: states of dead entries overwritten by a revival during the
// forward sweep; member b at offset b*cap
struct LogArr {
  uint64_t* key;  // determinant of the overwritten entry (the restore finds it through the index)
  uint32_t* meta;
  uint32_t* born;
  void* amp;
  uint64_t cap;
};

// per-step arrays (stride = max_factors + 1): scale/logn/logoff of member b
// at b*stride + k; the sharded accumulators pw/pcnt/gacc at
// (b*SH + shard)*stride + k, so different shards live in different lines.
struct StepArr {
  double* scale;   // scale[j] = S after step j
  Fx3* pw;         // removed raw weight at step k
  uint32_t* pcnt;  // removed count at step k
  Fx3* gacc;       // gradient dot product of step k
  uint32_t* logn;  // log records pushed at step k
  uint32_t* logoff;
  uint32_t* rmax;  // max over the batch of logn at step k (index k only)
  unsigned long long* ws;  // per-wave forward statistics, WSTAT per wave, nws waves per state
  int64_t nws;
  int64_t stride;
  // entropy tracking (null when off): sum r^2 ln r^2 and sum r^2 over the
  // live raw amplitudes r after step k, ES shards each at (b*ES + shard)*stride + k;
  // ent[b*stride + k] the resulting entropy
  Fx3* ea;
  Fx3* eb;
  double* ent;
  // live determinants visited by forward step k (= live when it began),
  // sharded like pcnt; shard 0 at k = 0 holds the live count after the sweep
  // (null unless tracked)
  uint32_t* pvis;
  // entries per arena when the forward launch at step k began (NB_UNSET where
  // no launch began: the second step of a two-factor launch, or not run yet),
  // and the entries that launch appended: [(b*nstride + k)*NA + arena]; the
  // counts of a launch are those of the one before it plus its appends, and
  // nb[M + 1] holds the counts at the end of the sweep
  uint32_t* nb;
  uint32_t* app;
  int64_t nstride;  // max_factors + 3
};
constexpr int WSTAT = 8;
// table slots each lane of a one-factor sweep step loads per pass
constexpr int SCAN_U = 2;
constexpr int ES = 16;

// N_MAX / N_CUT truncation: radix selection state of one batch member.  The
// rank of an entry is the 96-bit (FP32) or 128-bit (FP64) number
// (|amp| bits, ~key): larger rank = larger |c|, then smaller determinant.
constexpr int TK_BITS = 12;              // digit width of one selection pass
constexpr int TK_BINS = 1 << TK_BITS;
struct TKState {
  unsigned long long pre_hi, pre_lo;  // selected leading digits (right-aligned 128-bit)
  unsigned long long remaining;       // entries still to keep among those matching the prefix
  int depth;                          // digits selected
  int done;                           // selection finished
  int nokill;                         // at most N_MAX live entries: nothing to remove
  int pad;
};
// Pass p histograms into hist[p % 3]; the pass after it (or the kill) makes
// the selection of pass p from it in every block, and the state after the
// selection of pass p is kept in st[p & 1] (rotating, so that no launch
// writes what its own blocks read).
struct alignas(256) TopK {
  unsigned int hist[3][TK_BINS];
  TKState st[2];
};

// one checkpoint: snapshot of the live (key, raw amplitude) pairs of every
// member after a forward step; member b's entries at b*cap, count[b] entries
// written (a count above cap means the snapshot did not fit)
struct Snap {
  uint64_t* key;
  void* amp;
  unsigned long long* count;
  uint64_t cap;
};

// compact copies of the live entries (energy / state export), member b at b*cs
struct Compact {
  uint64_t* key;
  double* amp;
  uint32_t* slot;  // entry id
  double* sig;
  uint64_t cs;     // stride per member (>= its entries)
};

// ---------------------------------------------------------------------------
// kernel launchers (swc_kernels.hip); all asynchronous on `st`.  Launches
// that scan the entries take a grid of NA * r blocks (r blocks per arena).
// ---------------------------------------------------------------------------
// an empty state: index cleared (t.H slots), arenas empty
// pf: the index's presence filter, cleared with it (none by default)
void launch_fill(const Tab& t, int B, hipStream_t st, const Pf& pf = Pf{});
// insert n determinants (member b's at b * stride; n_fixed < 0: member b's
// count is cnt[b].ncompact) into an empty state; nmax bounds the counts
template <class T>
void launch_insert_list(const Tab& t, Counters* cnt, const uint64_t* keys, const double* amps, int64_t n_fixed,
                        uint64_t stride, int64_t nmax, int B, hipStream_t st, const Pf& pf = Pf{});
// record `msg` as the calling thread's last error (swc_last_error); returns code
int report_error(int code, const char* msg);

// member 0 only: flag F_BAD_INPUT unless every key of the list just
// inserted is a determinant of nq qubits, indexed under its own entry, with a
// finite amplitude
void launch_check_list(const Tab& t, Counters* cnt, const uint64_t* keys, const double* amps, int64_t n, int nq,
                       hipStream_t st);
void launch_trig(const double* theta, Trig* trig, int64_t M, int64_t ld, int B, Counters* cnt, hipStream_t st);
template <class T>
void launch_sweep_begin(const Tab& t, const StepArr& sa, Counters* cnt, int64_t M, int B, int grid, hipStream_t st);
// fold the per-wave statistics into the counters and set the arena counts
// after the last step that ran (fold_only: a run of steps up to k_last, cut
// short where a growth check stopped it); unless fold_only, also the final
// scale S_M and the counts the reverse sweep starts from
void launch_sweep_end(const Tab& t, const StepArr& sa, Counters* cnt, int64_t M, int64_t k_last, int B,
                      const Sync* sy, int fold_only, hipStream_t st);
void launch_sync_reset(Sync* sy, int clear_timeout, hipStream_t st);
// co-resident blocks per CU of the persistent forward (which=0) / reverse (1)
// sweep, of the one-factor forward (2) / reverse (3) step kernels, and of the
// wide two-factor forward (5) / reverse (6) kernels
template <class T>
int resident_blocks_per_cu(int which);
template <class T>
hipError_t launch_fwd_sweep(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa,
                            Counters* cnt, const LogArr& lg, int k0, int k1, double thr, int prune_first, int log_on,
                            Sync* sy, int B, int grid, hipStream_t st);
template <class T>
hipError_t launch_rev_sweep(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa,
                            Counters* cnt, const LogArr& lg, int k_hi, int k_lo, Sync* sy, int B, int grid,
                            hipStream_t st);
// occ_lim: a step whose start finds a member's entries above it does not run
// and stops the sweep (Counters::stop) so the host can grow the index;
// NO_LIMIT for an index at full capacity.  split: one launch per batch
// member (grid blocks each, one after the other) instead of one launch with
// grid.y = B.  hiocc: the forward build for more resident waves (large
// states; the entropy build has none).  pf.w set: the builds whose probes
// consult the index's presence filter first and keep it (not with entropy)
template <class T>
void launch_fwd(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                const LogArr& lg, int k, double thr, int prune_all, int log_on, uint64_t occ_lim, int B, int grid,
                int split, int hiocc, const Pf& pf, hipStream_t st);
template <class T>
void launch_rev(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                int k, int B, int grid, int split, const Pf& pf, hipStream_t st);
// steps k and k+1 in one launch (threshold 0, factors with different XOR
// masks; the index cannot grow during it), and their reverse (no truncation
// log) (wide: several index slots from every home loaded up front; for
// launches that cover the state in one pass with all blocks resident)
template <class T>
void launch_fwd2(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                 int k, int B, int grid, int wide, hipStream_t st);
template <class T>
void launch_rev2(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                 int k, int B, int grid, int wide, hipStream_t st);
template <class T>
void launch_log_restore(const Tab& t, const LogArr& lg, const StepArr& sa, int k, int B, uint32_t maxcnt,
                        hipStream_t st);
template <class T>
void launch_compact(const Tab& t, const Compact& cp, Counters* cnt, int B, int grid, hipStream_t st);
template <class T>
void launch_sigma(const Tab& t, const Compact& cp, const Counters* cnt, const double* h1, const double* h2, int nq,
                  int64_t nmax, int B, int singles_only, hipStream_t st);
// the off-diagonal part of sigma by pairing determinants on keys with `order`
// electrons removed (2: the doubles, 1: the singles; records (K, i) of one
// hash partition, radix-sorted by K); H is the stride of the compact arrays
void launch_pair_emit(const Compact& cp, uint64_t H, int b, uint64_t N, int part, int nparts, uint64_t* rk,
                      uint32_t* ri, unsigned long long* count, uint64_t cap, int order, hipStream_t st);
int launch_radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint64_t n, int bits, uint32_t* hist,
                      uint32_t* sums, hipStream_t st);
void launch_pair_groups(const Compact& cp, uint64_t H, int b, const uint64_t* K, const uint32_t* ri, uint64_t n,
                        uint64_t* rI, double* rc, const double* h1, const double* h2, int n_orb, Fx3* acc,
                        int order, hipStream_t st);
void launch_pair_finish(const Compact& cp, uint64_t H, int b, uint64_t N, Fx3* acc, hipStream_t st);
void launch_fx3_zero(Fx3* a, uint64_t n, hipStream_t st);
void launch_energy_reduce(const Compact& cp, Counters* cnt, const double* h1, const double* h2, int n, int64_t nmax,
                          int B, hipStream_t st);
void launch_energy_final(Counters* cnt, double* E, int B, hipStream_t st);
template <class T>
void launch_lambda(const Tab& t, const Compact& cp, const Counters* cnt, int64_t nmax, int B, hipStream_t st);
void launch_counters_reset(Counters* cnt, int B, double S0, hipStream_t st);
void launch_energy_begin(Counters* cnt, int B, hipStream_t st);
// zero the live and entry counts (before a state is refilled)
void launch_counters_live_reset(Counters* cnt, int B, hipStream_t st);
// entry positions the last sweeps of M factors scanned, into C_FSCAN / C_RSCAN
void launch_scan_totals(const StepArr& sa, Counters* cnt, int64_t M, int B, hipStream_t st);
// rebuild the index (t.H slots) from the entries; the growth stop is lifted
template <class T>
void launch_reindex(const Tab& t, Counters* cnt, int B, int grid, hipStream_t st, const Pf& pf = Pf{});
// the presence filter rebuilt from every member's entries
template <class T>
void launch_pf_build(const Tab& t, const Pf& pf, int B, int grid, hipStream_t st);
void launch_grad_final(const StepArr& sa, const Counters* cnt, double* grad, int64_t M, int B, hipStream_t st);
// checkpoints: write the live entries after step k into `sn` (count must be
// zero), and write a snapshot's amplitudes back over the entries of the same keys
template <class T>
void launch_snapshot(const Tab& t, const StepArr& sa, const Snap& sn, int k, int B, int grid, hipStream_t st);
template <class T>
void launch_snap_restore(const Tab& t, const Snap& sn, Counters* cnt, uint64_t nmax, int B, hipStream_t st);
void launch_zero_u64(unsigned long long* p, uint64_t n, hipStream_t st);
// N_MAX / N_CUT after forward step k: the selection passes and the removal
// (kernels only, so a captured graph may hold them); tk must start zeroed
template <class T>
void launch_topk(const Tab& t, const StepArr& sa, Counters* cnt, TopK* tk, int k, uint64_t n_max, uint64_t n_cut,
                 int B, int grid, hipStream_t st);
// entropy tracking: add the live entries of the state to step k's sums;
// turn the sums of steps 0..M into entropies
template <class T>
void launch_entropy_scan(const Tab& t, const StepArr& sa, int k, int B, int grid, hipStream_t st);
void launch_entropy_final(const StepArr& sa, int64_t M, int B, hipStream_t st);

int grid_for(uint64_t work, int block, int cap);

}  // namespace swc
