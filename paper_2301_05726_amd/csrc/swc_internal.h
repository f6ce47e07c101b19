// Internal definitions shared by the kernels (swc_kernels.hip) and the host
// side of the C ABI (swc_api.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace swc {

// ---------------------------------------------------------------------------
// hash-table slot encoding
// ---------------------------------------------------------------------------
// keys[s] == EMPTY_KEY: never used.  Otherwise meta[s] holds a state bit and
// a step tag (1-based factor index within the current sweep, 0 = before it):
//   alive:  meta = born tag          (step that created the entry)
//   dead:   meta = DEAD | death tag   (step whose truncation removed it)
// born[s] keeps the creation tag of dead entries (needed when the reverse
// sweep resurrects them).  A dead entry keeps its key (tombstone) and, for a
// death during the current sweep, the pre-truncation amplitude.
constexpr uint64_t EMPTY_KEY = ~0ull;
constexpr uint64_t NO_LIMIT = ~0ull;  // occupancy limit of a table that cannot grow
constexpr int SH = 64;  // shards of each per-step accumulator
constexpr uint32_t DEAD = 0x80000000u;
constexpr uint32_t TAG = 0x7fffffffu;

// status flags (Counters::flags)
enum : uint32_t {
  F_TABLE_FULL = 1u,
  F_LOG_FULL = 2u,
  F_BAD_THETA = 4u,
  F_INCONSISTENT = 8u,
  F_TIMEOUT = 16u,  // a grid barrier of a persistent sweep gave up waiting
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
  C_OCC,       // slots holding a key (alive + tombstones)
  C_DU,        // det visits (forward)
  C_PAIRS,     // rotated pairs (forward)
  C_INS,       // created entries (forward)
  C_PRUNED,    // truncated amplitudes (forward)
  C_HITS,      // rotated pairs whose partner existed (forward)
  C_COPY,      // slots copied by the last rehash
  C_NCNT
};
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

// Hash-table slots.  float states: 16-byte {key, amp, meta} plus an 8-byte
// side array {lam, born}; double states: one 32-byte slot.  lam is the
// adjoint amplitude of the reverse sweep, born the creation tag.
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

// per-state tables; member b's slots start at b*H
struct Tab {
  void* slots;  // Slot<T>[B*H]
  void* aux;    // AuxF[B*H] for float states, unused for double
  uint64_t H;   // slots per state, power of two
};

// truncation log: states of tombstones overwritten by a resurrection
// during the forward sweep; member b at offset b*cap
struct LogArr {
  uint64_t* key;  // determinant of the overwritten tombstone (slots move on a rehash)
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

// compact copies of the live entries (energy / state export), member b at b*H
struct Compact {
  uint64_t* key;
  double* amp;
  uint32_t* slot;
  double* sig;
};

// ---------------------------------------------------------------------------
// kernel launchers (swc_kernels.hip); all asynchronous on `st`
// ---------------------------------------------------------------------------
template <class T>
void launch_fill(const Tab& t, int B, hipStream_t st);
template <class T>
void launch_insert_init(const Tab& t, Counters* cnt, const uint64_t* dets, const double* amps, int64_t n, int B,
                        hipStream_t st);
void launch_trig(const double* theta, Trig* trig, int64_t M, int64_t ld, int B, Counters* cnt, hipStream_t st);
template <class T>
void launch_sweep_begin(const Tab& t, const StepArr& sa, Counters* cnt, int64_t M, int B, hipStream_t st);
// fold the per-wave statistics into the counters; unless fold_only, also the
// final scale S_M
void launch_sweep_end(const StepArr& sa, Counters* cnt, int64_t M, int B, const Sync* sy, int fold_only,
                      hipStream_t st);
void launch_sync_reset(Sync* sy, int clear_timeout, hipStream_t st);
// co-resident blocks per CU of the persistent forward (which=0) / reverse (1)
// sweep, and of the one-factor forward (2; 4: the five-wave build) / reverse
// (3) step kernels
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
// occ_lim: a step that sees a member's occupancy above it stops the steps
// after the next one (Counters::stop) so the host can grow the table;
// NO_LIMIT for a table at full capacity.  wide: the kernel built for five
// resident waves per SIMD (tables scanned in many passes)
template <class T>
void launch_fwd(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                const LogArr& lg, int k, double thr, int prune_all, int log_on, uint64_t occ_lim, int B, int grid,
                int wide, hipStream_t st);
template <class T>
void launch_rev(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                int k, int B, int grid, hipStream_t st);
// steps k and k+1 in one launch (threshold 0, factors with different XOR
// masks; the table cannot grow during it), and their reverse (no truncation log)
// (wide: several slots from every home loaded up front; for launches that
// cover the table in one pass with all blocks resident)
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
// sigma of double excitations by pairing determinants on two-electron-removed
// keys (records (K, i) of one hash partition, radix-sorted by K)
void launch_pair_emit(const Compact& cp, uint64_t H, int b, uint64_t N, int part, int nparts, uint64_t* rk,
                      uint32_t* ri, unsigned long long* count, uint64_t cap, hipStream_t st);
int launch_radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint64_t n, int bits, uint32_t* hist,
                      uint32_t* sums, hipStream_t st);
void launch_pair_groups(const Compact& cp, uint64_t H, int b, const uint64_t* K, const uint32_t* ri, uint64_t n,
                        uint64_t* rI, double* rc, const double* h1, const double* h2, int n_orb, Fx3* acc,
                        hipStream_t st);
void launch_pair_finish(const Compact& cp, uint64_t H, int b, uint64_t N, Fx3* acc, hipStream_t st);
void launch_fx3_zero(Fx3* a, uint64_t n, hipStream_t st);
void launch_energy_reduce(const Compact& cp, Counters* cnt, uint64_t H, const double* h1, const double* h2, int n,
                          int64_t nmax, int B, hipStream_t st);
void launch_energy_final(Counters* cnt, double* E, int B, hipStream_t st);
template <class T>
void launch_lambda(const Tab& t, const Compact& cp, const Counters* cnt, int64_t nmax, int B, hipStream_t st);
void launch_counters_reset(Counters* cnt, int B, double S0, hipStream_t st);
void launch_energy_begin(Counters* cnt, int B, hipStream_t st);
// rehash every slot of `from` that is alive or a tombstone with a step tag in
// [1, tag_max] into the table `to` (cleared first; larger when the forward
// sweep grows, smaller when the reverse sweep shrinks); the occupancy counter
// becomes the number of slots copied
template <class T>
void launch_rehash(const Tab& from, const Tab& to, Counters* cnt, int B, uint32_t tag_max, hipStream_t st);
// number of slots such a rehash would copy, into the C_COPY counters
template <class T>
void launch_count_keep(const Tab& t, Counters* cnt, int B, uint32_t tag_max, hipStream_t st);
void launch_grad_final(const StepArr& sa, const Counters* cnt, double* grad, int64_t M, int B, hipStream_t st);
// checkpoints: write the live entries into `sn` (count must be zero), and
// write a snapshot's amplitudes back over the entries of the same keys
template <class T>
void launch_snapshot(const Tab& t, const Snap& sn, int B, int grid, hipStream_t st);
template <class T>
void launch_snap_restore(const Tab& t, const Snap& sn, Counters* cnt, uint64_t nmax, int B, hipStream_t st);
void launch_zero_u64(unsigned long long* p, uint64_t n, hipStream_t st);
// N_MAX / N_CUT after forward step k: the selection passes and the removal
// (kernels only, so a captured graph may hold them); tk must start zeroed
template <class T>
void launch_topk(const Tab& t, const StepArr& sa, Counters* cnt, TopK* tk, int k, uint64_t n_max, uint64_t n_cut,
                 int B, int grid, hipStream_t st);
// entropy tracking: add the live entries of the table to step k's sums;
// turn the sums of steps 0..M into entropies
template <class T>
void launch_entropy_scan(const Tab& t, const StepArr& sa, int k, int B, int grid, hipStream_t st);
void launch_entropy_final(const StepArr& sa, int64_t M, int B, hipStream_t st);

int grid_for(uint64_t work, int block, int cap);

}  // namespace swc
