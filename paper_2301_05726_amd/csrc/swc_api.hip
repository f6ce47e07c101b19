// Host side of the C ABI declared in include/swc.h: argument checks,
// workspace carving, and the orchestration of the forward sweep, the energy
// and the adjoint sweep on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_set>
#include <utility>
#include <vector>

#include "swc.h"
#include "swc_internal.h"

using namespace swc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

int swc::report_error(int code, const char* msg) { return fail(code, msg); }

namespace {

#define SWC_HIP(call)                                                                                    \
  do {                                                                                                   \
    hipError_t e_ = (call);                                                                              \
    if (e_ != hipSuccess) return fail(SWC_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_));     \
  } while (0)

constexpr size_t ALIGN = 256;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Byte offsets of every workspace region.
struct Layout {
  size_t ent, aux, idx, ac;
  size_t lkey, lmeta, lborn, lamp;
  size_t scale, pw, pcnt, gacc, logn, logoff, rmax, ws, ea, eb, entr, pvis, nb, app;
  size_t ckey, camp, cslot, csig;
  size_t cnt, fac, trig, init_d, init_a, sync, topk, pf;
  size_t total;
};

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

// Sweep kernels use at most this many 256-thread blocks per state (NA-way
// interleaved over the arenas); each of their waves owns a statistics slot.
constexpr int MAX_SWEEP_BLOCKS = 2048;
constexpr int MAX_ARENA_BLOCKS = MAX_SWEEP_BLOCKS / NA;
size_t max_waves() { return static_cast<size_t>(MAX_SWEEP_BLOCKS) * 4; }

// Entries per arena for an index of Hcap slots: an even share of 90% of
// Hcap.  The arenas bound the index's occupancy at full size, where no growth
// check runs: an entry that finds its arena full fails the sweep with
// "hash table full" before the index passes about 90% (past that, a linear
// probe for an absent key grows without bound).
uint64_t arena_size(uint64_t Hcap) {
  const uint64_t a = Hcap / 10 * 9 / NA + 64;
  return std::min<uint64_t>(a, 1ull << ID_POS_BITS);
}

Layout make_layout(uint64_t Hcap, int tsz, int B, int64_t Mmax, uint64_t L) {
  Layout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t BE = static_cast<size_t>(B) * NA * arena_size(Hcap);
  const size_t BH = static_cast<size_t>(B) * Hcap;
  const size_t BL = static_cast<size_t>(B) * L;
  const size_t BS = static_cast<size_t>(B) * static_cast<size_t>(Mmax + 1);
  l.ent = take(BE * (tsz == 4 ? sizeof(Slot<float>) : sizeof(Slot<double>)));
  l.aux = take(tsz == 4 ? BE * sizeof(AuxF) : 0);
  l.idx = take(BH * sizeof(Idx));
  l.ac = take(static_cast<size_t>(B) * NA * 4);
  l.lkey = take(BL * 8);
  l.lmeta = take(BL * 4);
  l.lborn = take(BL * 4);
  l.lamp = take(BL * tsz);
  l.scale = take(BS * 8);
  l.pw = take(BS * SH * sizeof(Fx3));
  l.pcnt = take(BS * SH * 4);
  l.gacc = take(BS * SH * sizeof(Fx3));
  l.logn = take(BS * 4);
  l.logoff = take(BS * 4);
  l.rmax = take(static_cast<size_t>(Mmax + 1) * 4);
  l.ws = take(static_cast<size_t>(B) * max_waves() * WSTAT * 8);
  l.ea = take(BS * ES * sizeof(Fx3));
  l.eb = take(BS * ES * sizeof(Fx3));
  l.entr = take(BS * 8);
  l.pvis = take(BS * SH * 4);
  l.nb = take(static_cast<size_t>(B) * static_cast<size_t>(Mmax + 3) * NA * 4);
  l.app = take(static_cast<size_t>(B) * static_cast<size_t>(Mmax + 3) * NA * 4);
  l.ckey = take(BE * 8);
  l.camp = take(BE * 8);
  l.cslot = take(BE * 4);
  l.csig = take(BE * 8);
  l.cnt = take(static_cast<size_t>(B) * sizeof(Counters));
  l.fac = take(static_cast<size_t>(Mmax + 1) * sizeof(FacMask));
  l.trig = take(static_cast<size_t>(B) * static_cast<size_t>(Mmax + 1) * sizeof(Trig));
  l.init_d = take(Hcap / 2 * 8);
  l.init_a = take(Hcap / 2 * 8);
  l.sync = take(sizeof(Sync));
  l.topk = take(static_cast<size_t>(B) * sizeof(TopK));
  l.pf = take(BH);  // presence filter: one 64-bit word per 8 index slots
  l.total = off;
  return l;
}

uint64_t btw(int lo, int hi) {  // bits strictly between lo and hi (lo < hi)
  uint64_t upto_hi = (hi >= 64) ? ~0ull : ((1ull << hi) - 1ull);
  uint64_t thru_lo = (lo >= 63) ? ~0ull : ((2ull << lo) - 1ull);
  return upto_hi & ~thru_lo;
}

int check_exc(int nq, const swc_exc* exc, int64_t M) {
  if (M < 0) return fail(SWC_EINVAL, "negative factor count");
  if (M > 0 && !exc) return fail(SWC_EINVAL, "null excitation list");
  for (int64_t k = 0; k < M; ++k) {
    const swc_exc& e = exc[k];
    char buf[128];
    std::snprintf(buf, sizeof buf, "invalid excitation %lld = (%d,%d,%d,%d)", static_cast<long long>(k), e.i, e.j,
                  e.a, e.b);
    if (e.j == -1 && e.b == -1) {
      if (e.i < 0 || e.a < 0 || e.i >= nq || e.a >= nq || e.i == e.a) return fail(SWC_EINVAL, buf);
      continue;
    }
    if (e.i < 0 || e.j < 0 || e.a < 0 || e.b < 0) return fail(SWC_EINVAL, buf);
    if (e.i >= nq || e.j >= nq || e.a >= nq || e.b >= nq) return fail(SWC_EINVAL, buf);
    if (!(e.i < e.j) || !(e.a < e.b)) return fail(SWC_EINVAL, buf);
    if (e.i == e.a || e.i == e.b || e.j == e.a || e.j == e.b) return fail(SWC_EINVAL, buf);
  }
  return SWC_OK;
}

// Occupied-side, virtual-side and sign masks of one factor.  Sign rule: for
// tau = a+_a a+_b a_j a_i on the lower determinant L the Jordan-Wigner phase
// is the parity of the occupied orbitals strictly between i and j plus those
// strictly between a and b after i, j are emptied; bits of the four moved
// orbitals are removed so the same mask serves the upper member.  A single
// a+_a a_i counts the occupied orbitals strictly between i and a.
FacMask factor_mask(const swc_exc& e) {
  FacMask f;
  if (e.j == -1 && e.b == -1) {
    f.occ = 1ull << e.i;
    f.vir = 1ull << e.a;
    const int lo = std::min<int>(e.i, e.a), hi = std::max<int>(e.i, e.a);
    f.sgn = btw(lo, hi) & ~(f.occ | f.vir);
  } else {
    f.occ = (1ull << e.i) | (1ull << e.j);
    f.vir = (1ull << e.a) | (1ull << e.b);
    f.sgn = (btw(e.i, e.j) ^ (btw(e.a, e.b) & ~f.occ)) & ~(f.occ | f.vir);
  }
  return f;
}

// A captured run of per-step kernels: direction (0 forward, 1 reverse),
// steps k0..k1, threshold, log flag, index size, occupancy limit and the optional
// per-step arrays are baked into the kernel arguments; the choice of fused
// factor pairs depends on the excitation list, whose upload clears the cache.
struct GraphKey {
  int dir;
  int64_t k0, k1;
  double thr;
  int log_on;
  uint64_t H, lim;
  int ent = 0;
  uint64_t tk_max = 0, tk_cut = 0;
  int live = 0;  // the live-count array is passed to the kernels (swc_track_live)
  int pf = 0;    // the one-factor steps probe through the presence filter
  bool operator==(const GraphKey& o) const {
    return dir == o.dir && k0 == o.k0 && k1 == o.k1 && thr == o.thr && log_on == o.log_on &&
           H == o.H && lim == o.lim && ent == o.ent && tk_max == o.tk_max && tk_cut == o.tk_cut && live == o.live &&
           pf == o.pf;
  }
};
constexpr int64_t GRAPH_CHUNK = 2048;
constexpr size_t GRAPH_CACHE_MAX = 512;  // executable graphs kept per context
constexpr uint64_t RS_CAP_SLACK = 4096;  // records kept below the sort's 2^28 limit

// Steps run in chunks [2^(j-1) + 1, 2^j] up to GRAPH_CHUNK and in chunks
// [m GRAPH_CHUNK + 1, (m + 1) GRAPH_CHUNK] above (so a chunk ends at every
// power of two up to GRAPH_CHUNK and at every multiple of it).
int64_t chunk_end(int64_t k) {
  if (k > GRAPH_CHUNK) return (k + GRAPH_CHUNK - 1) / GRAPH_CHUNK * GRAPH_CHUNK;
  int64_t p = 1;
  while (p < k) p *= 2;
  return p;
}

}  // namespace

struct swc_ctx {
  int nq = 0, na = 0, nb = 0, prec = 0, B = 1;
  uint64_t H = 0, L = 0;  // H: capacity (largest index), L: log records per state
  // The index starts small and is rebuilt larger from the entries (which never
  // move) between chunks of steps.  Smallest index after a reset
  // (SWC_TABLE_MIN): 2^18 slots, so that growing below that adds no host
  // round trips.
  uint64_t table_min = 1ull << 18;
  int grid_override = 0;       // SWC_GRID
  int split_override = -1;     // SWC_SPLIT: 1 members always launched apart, 0 never, unset by index size
  int hiocc_override = -1;     // SWC_HIOCC: 1 forward steps always on their high-occupancy build, 0 never, unset by index size
  // Probes through the index's presence filter (SWC_PFILTER: 1 always, 0
  // never; unset: unless the last completed forward sweep found the partner
  // of more than 1 rotated pair in 4, where most probes would read the
  // filter and then the index anyway).  pf_now: the choice for the current
  // call's sweeps; pf_fwd / pf_rev: whether the forward range being issued /
  // the reverse sweep probe through it (forward ranges only on indexes of
  // PF_FWD_H slots and more).
  int pf_override = -1;
  bool pf_auto = true, pf_now = false, pf_fwd = false, pf_rev = false;
  Pf pf;                  // the filter (one word per 8 index slots of every member)
  bool pf_valid = false;  // it holds every indexed key (steps without it leave it stale)
  // two factors per launch at threshold 0 (SWC_FUSE=0 turns it off)
  bool fuse = true;
  // entropy of every forward step (swc_track_entropy); sa.ea/eb are set
  // while it is on; ent_M: factors of the last tracked sweep (-1: none)
  bool entropy = false;
  Fx3* ent_ea = nullptr;
  Fx3* ent_eb = nullptr;
  int64_t ent_M = -1;
  // live count before every forward step (swc_track_live): sa.pvis is set
  // while it is on; live_M: factors of the last tracked sweep (-1: none)
  bool live = false;
  uint32_t* live_pvis = nullptr;
  int64_t live_M = -1;
  // sigma of doubles by pairing (swc_set_sigma_scratch): caller's scratch;
  // mode 0 auto, 1 always, 2 never (probes)
  char* sig_buf = nullptr;
  size_t sig_bytes = 0;
  int sig_mode = 2;
  int64_t sig_parts = 0;  // partitions used by the last pairing sigma (0: probes)
  // N_MAX / N_CUT truncation after every factor (swc_set_topk; 0 = off)
  uint64_t tk_max = 0, tk_cut = 0;
  TopK* tk = nullptr;
  std::vector<uint64_t> hmask;  // XOR mask (occ | vir) of every uploaded factor
  // checkpoints (swc_set_checkpoints): snapshot j holds the state after
  // forward step (j + 1) * ck_interval, in a caller-owned buffer
  int64_t ck_interval = 0;
  uint64_t ck_cap = 0;
  int64_t ck_n = 0;  // snapshots the buffer holds
  uint64_t* ck_key = nullptr;
  char* ck_amp = nullptr;
  unsigned long long* ck_count = nullptr;
  int64_t ck_taken = 0;
  std::vector<uint64_t> ck_nmax;  // per checkpoint: most entries over the batch (last sweep)
  int64_t fwd_launches = 0, rev_launches = 0;  // launches of the last sweeps (per-launch timing)
  int64_t rehashes = 0;        // index rebuilds (growths) in the last forward sweep
  int64_t compactions = 0;     // rebuilds without the dead entries of earlier sweeps at its start
  int64_t last_M = 0;          // factors of the last forward sweep (entry-scan totals of swc_get_stats)
  bool rev_fused = false;      // the last reverse sweep undid two factors per launch
  int64_t builds = 0;          // SWC_BUILD_* bits of the kernels the last sweeps launched
  int64_t Mmax = 0;
  hipStream_t st = nullptr;
  char* ws = nullptr;
  Layout lay{};
  Tab tab{};
  LogArr lg{};
  StepArr sa{};
  Compact cp{};
  Counters* cnt = nullptr;
  FacMask* fac = nullptr;
  Trig* trig = nullptr;
  uint64_t* init_d = nullptr;
  double* init_a = nullptr;
  std::vector<uint64_t> h_init_d;
  std::vector<double> h_init_a;
  double S0 = 1.0;
  bool built = false;
  bool fresh = false;  // the table holds |Psi_0> exactly as a reset leaves it (no call since)
  std::vector<swc_exc> exc_cache;
  hipEvent_t ev[8] = {};
  double fwd_ms = 0, energy_ms = 0, rev_ms = 0;
  int64_t log_records = 0;
  // Launches that scan the entries take NA * r blocks (r per arena).  grid:
  // one entry per lane for the entries the current index may hold at its
  // growth limit (the two-factor kernels and the one-pass kernels).  The
  // one-factor step kernels are latency-bound while the state is small: they
  // run fastest with as many lanes as can be resident at once (one wave
  // round, the SCAN_U entries of a lane loaded together), and no more.
  // res_fwd / res_rev: resident blocks of k_fwd / k_rev on the whole device.
  int grid = NA;
  int grid_fs = NA, grid_rs = NA;
  int res_fwd = 0, res_rev = 0;
  // the same for launches of one batch member each (split_members)
  int grid_fs1 = NA, grid_rs1 = NA;
  int res_fwd1 = 0, res_rev1 = 0;
  // the same for the forward build with more resident waves (hi_occ), all
  // members in one launch and one member per launch
  int grid_fsh = NA, grid_fsh1 = NA;
  int res_fwdh = 0, res_fwdh1 = 0;
  int res_f2w = 0, res_r2w = 0;  // resident blocks (all members) of the wide two-factor kernels
  uint64_t per_arena = 0;  // entries per arena the grids are sized for
  // persistent (cooperative) sweeps, one launch per sweep: opt-in with
  // SWC_SWEEP=persistent (per-step launches are faster on MI355X: a
  // device-wide barrier needs agent-scope fences in every block)
  bool persistent = false;
  Sync* sy = nullptr;
  int grid_fwd = 1, grid_rev = 1;
  std::vector<Counters> hcnt;
  // per-step sweeps replayed from captured hipGraphs (SWC_GRAPH=0 disables)
  bool use_graph = true;
  // SWC_PROGRESS=1: after each range of steps, wait for it and report it on
  // stderr (long sweeps at large sizes; off by default: it adds a host wait)
  bool progress = false;
  hipStream_t cap_st = nullptr;
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
  // optional per-launch timing (SWC_KERNEL_TIMING=1)
  bool ktiming = false;
  std::vector<hipEvent_t> kev;
  double rot_ms = 0, revk_ms = 0, sig_ms = 0;
  int64_t grad_calls = 0;  // completed energy_and_grad calls, and their summed sweep and sigma times
  double fwd_ms_total = 0, rev_ms_total = 0, sig_ms_total = 0;
  int64_t rot_n = 0, revk_n = 0;
};

namespace {

template <class F>
int dispatch(swc_ctx* c, F&& f) {
  if (c->prec == SWC_FP32) return f(static_cast<float*>(nullptr));
  return f(static_cast<double*>(nullptr));
}

int read_counters(swc_ctx* c) {
  SWC_HIP(hipMemcpyAsync(c->hcnt.data(), c->cnt, sizeof(Counters) * c->B, hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipStreamSynchronize(c->st));
  return SWC_OK;
}

int upload_masks(swc_ctx* c, const swc_exc* exc, int64_t M) {
  if (M == 0) return SWC_OK;
  if (static_cast<int64_t>(c->exc_cache.size()) == M &&
      std::memcmp(c->exc_cache.data(), exc, sizeof(swc_exc) * M) == 0)
    return SWC_OK;
  std::vector<FacMask> f(static_cast<size_t>(M));
  c->hmask.resize(static_cast<size_t>(M));
  for (int64_t k = 0; k < M; ++k) {
    f[k] = factor_mask(exc[k]);
    c->hmask[k] = f[k].occ | f[k].vir;
  }
  SWC_HIP(hipMemcpyAsync(c->fac, f.data(), sizeof(FacMask) * M, hipMemcpyHostToDevice, c->st));
  SWC_HIP(hipStreamSynchronize(c->st));
  c->exc_cache.assign(exc, exc + M);
  // Captured sweeps bake in which neighbouring factors share a launch (a
  // choice made from the XOR masks): graphs recorded for another list are
  // dropped (the stream has just been synchronized, so none is running).
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  c->graphs.clear();
  return SWC_OK;
}

// A grid of NA * r blocks, r blocks of 256 lanes per arena covering `per`
// entries of an arena `items` per lane, at least 1 and at most rmax blocks
// per arena.
int arena_grid(uint64_t per, int items, int rmax) {
  uint64_t r = (per + 256 * items - 1) / (256 * items);
  r = std::max<uint64_t>(1, std::min<uint64_t>(r, static_cast<uint64_t>(std::max(1, rmax))));
  return static_cast<int>(r) * NA;
}

// Make an index of Hn slots the current one (the grids follow its size).
void set_table(swc_ctx* c, uint64_t Hn) {
  c->tab.H = Hn;
  c->pf.n = Hn / 8;  // the presence filter follows the index
  // the entries an index of Hn slots holds when it runs at 45%, per arena
  c->per_arena = (Hn / 20 * 9 + NA - 1) / NA;
  int rmax = MAX_ARENA_BLOCKS;
  if (c->grid_override > 0) rmax = std::max(1, c->grid_override / NA);
  c->grid = arena_grid(c->per_arena, 1, rmax);
  c->grid_fs = arena_grid(c->per_arena, SCAN_U, std::min(rmax, c->res_fwd > 0 ? c->res_fwd / NA : rmax));
  c->grid_rs = arena_grid(c->per_arena, SCAN_U, std::min(rmax, c->res_rev > 0 ? c->res_rev / NA : rmax));
  c->grid_fs1 = arena_grid(c->per_arena, SCAN_U, std::min(rmax, c->res_fwd1 > 0 ? c->res_fwd1 / NA : rmax));
  c->grid_rs1 = arena_grid(c->per_arena, SCAN_U, std::min(rmax, c->res_rev1 > 0 ? c->res_rev1 / NA : rmax));
  c->grid_fsh = arena_grid(c->per_arena, SCAN_U, std::min(rmax, c->res_fwdh > 0 ? c->res_fwdh / NA : rmax));
  c->grid_fsh1 = arena_grid(c->per_arena, SCAN_U, std::min(rmax, c->res_fwdh1 > 0 ? c->res_fwdh1 / NA : rmax));
}

// Batch members get one-factor step launches of their own once their indexes
// are large (64 MiB and more each): a launch then works on one member's index
// and entries instead of all B members' at once, which would share the L2 and
// Infinity Cache between them.  Small states keep one launch for all members
// (latency-bound launches, where fewer launches win).
constexpr uint64_t SPLIT_H = 1ull << 22;
bool split_members(const swc_ctx* c) {
  return c->B > 1 && (c->split_override >= 0 ? c->split_override > 0 : c->tab.H >= SPLIT_H);
}
// The one-factor forward steps use their build for more resident waves once
// the index reaches 2^22 slots (a state of a million entries and more: many
// passes of the grid per step, where more loads in flight per compute unit
// pay); below, the launches are short dependent chains and the lighter
// build is faster.
constexpr uint64_t HIOCC_H = 1ull << 22;
bool hi_occ(const swc_ctx* c) {
  return c->hiocc_override >= 0 ? c->hiocc_override > 0 : c->tab.H >= HIOCC_H;
}
// The filter the one-factor step launches probe through (none: plain
// probes).  Forward steps use it from PF_FWD_H index slots on: on smaller
// indexes a forward launch is a short chain of dependent loads that the
// filter's second round trip (for the few partners it may hold, and for the
// pairs that create their partner) lengthens, while the reverse, which
// creates nothing, gains at every size.
constexpr uint64_t PF_FWD_H = 1ull << 22;
Pf fwd_pf(const swc_ctx* c) { return c->pf_fwd ? c->pf : Pf{}; }
Pf rev_pf(const swc_ctx* c) { return c->pf_rev ? c->pf : Pf{}; }

// Keys enter the index without their filter bits in forward ranges that do
// not use the filter; the filter is rebuilt from the entries before it is
// used again (a growth's rebuild of the index rebuilds it too).
template <class T>
void pf_ensure(swc_ctx* c) {
  if (c->pf_valid) return;
  launch_pf_build<T>(c->tab, c->pf, c->B, c->grid, c->st);
  c->pf_valid = true;
}
void pf_ensure_any(swc_ctx* c) {
  dispatch(c, [&](auto* tp) -> int {
    pf_ensure<std::remove_pointer_t<decltype(tp)>>(c);
    return SWC_OK;
  });
}

int fwd_grid(const swc_ctx* c) {
  if (hi_occ(c)) return split_members(c) ? c->grid_fsh1 : c->grid_fsh;
  return split_members(c) ? c->grid_fs1 : c->grid_fs;
}
int rev_grid(const swc_ctx* c) { return split_members(c) ? c->grid_rs1 : c->grid_rs; }
int64_t step_launches(const swc_ctx* c) { return split_members(c) ? c->B : 1; }

// Two-factor launches load several index slots per probe up front when one
// launch covers the state in one pass and all its blocks are resident at once.
int wide2(const swc_ctx* c, int resident) {
  return static_cast<uint64_t>(c->grid / NA) * 256 >= c->per_arena &&
         static_cast<int64_t>(c->grid) * c->B <= static_cast<int64_t>(resident);
}

// Entries above which a forward step does not run and stops the sweep for a
// growth of the index: a step that runs at most doubles the entries, so the
// index never passes 2 x 0.225 = 45% occupancy.  (The index is only probed,
// never scanned: a sparser one costs memory, not scan time, and its probes
// end in the first slots loaded.)
uint64_t occ_limit(const swc_ctx* c) { return c->tab.H < c->H ? c->tab.H / 40 * 9 : NO_LIMIT; }

// Smallest index, at least Hmin, that holds `need` entries at <= 10% load.
uint64_t table_size_for(const swc_ctx* c, uint64_t need, uint64_t Hmin) {
  if (c->persistent) return c->H;  // a persistent sweep cannot stop for a growth
  uint64_t h = std::min(Hmin, c->H);
  while (h < c->H && need > h / 10) h <<= 1;
  return h;
}

// Rebuild the index with Hn slots from the entries (the arena counts are
// current: the sweep's runs end with a fold that sets them).
int reindex_to(swc_ctx* c, uint64_t Hn) {
  set_table(c, Hn);
  dispatch(c, [&](auto* tp) -> int {
    launch_reindex<std::remove_pointer_t<decltype(tp)>>(c->tab, c->cnt, c->B, c->grid, c->st, c->pf);
    return SWC_OK;
  });
  SWC_HIP(hipGetLastError());
  c->pf_valid = true;  // every entry's key re-entered the index and the filter
  ++c->rehashes;
  return SWC_OK;
}

// Grow the index (x2 at least) so that `need` entries stay under the growth
// limit of the new size.
int grow_table(swc_ctx* c, uint64_t need) {
  if (c->persistent || c->tab.H >= c->H) return SWC_OK;
  uint64_t Hn = 2 * c->tab.H;
  while (Hn < c->H && need > Hn / 40 * 9) Hn <<= 1;
  return reindex_to(c, std::min(Hn, c->H));
}

// Reset every batch member to |Psi_0> with an index sized for it.
int reset_state(swc_ctx* c) {
  set_table(c, table_size_for(c, c->h_init_d.size(), c->table_min));
  launch_fill(c->tab, c->B, c->st, c->pf);
  for (int b = 0; b < c->B; ++b) {
    Counters z{};
    z.S = c->S0;
    z.stop = ~0u;
    c->hcnt[b] = z;
  }
  // the device counters are set by a kernel and the initial determinants are
  // already on the device (copied by swc_build_state): a reset issues no copy
  // from pageable host memory, which would wait for the stream
  launch_counters_reset(c->cnt, c->B, c->S0, c->st);
  const int64_t n = static_cast<int64_t>(c->h_init_d.size());
  int r = dispatch(c, [&](auto* tp) -> int {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_insert_list<T>(c->tab, c->cnt, c->init_d, c->init_a, n, 0, n, c->B, c->st, c->pf);
    return SWC_OK;
  });
  if (r) return r;
  SWC_HIP(hipGetLastError());
  c->pf_valid = true;
  c->fresh = true;
  return SWC_OK;
}

// Drop the dead entries of earlier sweeps: the live entries are copied out
// (the compact arrays), the state is emptied and they are inserted again.
// Every live entry is tagged 0 at a sweep's start anyway.
int compact_state(swc_ctx* c, uint64_t live) {
  launch_energy_begin(c->cnt, c->B, c->st);
  int r = dispatch(c, [&](auto* tp) -> int {
    launch_compact<std::remove_pointer_t<decltype(tp)>>(c->tab, c->cp, c->cnt, c->B, c->grid, c->st);
    return SWC_OK;
  });
  if (r) return r;
  set_table(c, table_size_for(c, live, c->table_min));
  launch_fill(c->tab, c->B, c->st, c->pf);
  launch_counters_live_reset(c->cnt, c->B, c->st);
  r = dispatch(c, [&](auto* tp) -> int {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_insert_list<T>(c->tab, c->cnt, c->cp.key, c->cp.amp, -1, c->cp.cs, static_cast<int64_t>(live), c->B,
                          c->st, c->pf);
    return SWC_OK;
  });
  if (r) return r;
  SWC_HIP(hipGetLastError());
  c->pf_valid = true;
  return SWC_OK;
}

// Angles -> cos/sin table.  A non-finite angle sets F_BAD_THETA; with
// wait = false the caller reads that flag later with other counters (the
// sweep meanwhile runs on values it cannot overflow the table with: every
// comparison with a NaN amplitude removes it).
int check_theta(swc_ctx* c, const double* theta, int64_t M, bool wait = true) {
  if (M == 0) return SWC_OK;
  if (!theta) return fail(SWC_EINVAL, "null theta");
  launch_trig(theta, c->trig, M, c->Mmax + 1, c->B, c->cnt, c->st);
  SWC_HIP(hipGetLastError());
  if (!wait) return SWC_OK;
  int r = read_counters(c);
  if (r) return r;
  if (c->hcnt[0].flags & F_BAD_THETA) {
    unsigned int z = c->hcnt[0].flags & ~F_BAD_THETA;
    SWC_HIP(hipMemcpyAsync(&c->cnt[0].flags, &z, sizeof z, hipMemcpyHostToDevice, c->st));
    SWC_HIP(hipStreamSynchronize(c->st));
    return fail(SWC_EINVAL, "theta contains a non-finite value");
  }
  return SWC_OK;
}

// Event pool for per-launch timing: 2 events per timed launch.
int ensure_kev(swc_ctx* c, size_t n) {
  while (c->kev.size() < n) {
    hipEvent_t e;
    SWC_HIP(hipEventCreate(&e));
    c->kev.push_back(e);
  }
  return SWC_OK;
}

// Sum of the durations between event pairs [2i, 2i+1) for i < n.
double sum_pairs(swc_ctx* c, int64_t n) {
  double t = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->kev[2 * i], c->kev[2 * i + 1]) == hipSuccess) t += ms;
  }
  return t;
}

// Executable graph for `key`, captured on first use: `record(stream)` issues
// the kernel launches on a private capture stream (kernels only, no memset
// or copy nodes); the graph is then replayed on the caller's stream.
template <class F>
int cached_graph(swc_ctx* c, const GraphKey& key, hipGraphExec_t* out, F&& record) {
  for (auto& g : c->graphs)
    if (g.first == key) {
      *out = g.second;
      return SWC_OK;
    }
  if (c->graphs.size() >= GRAPH_CACHE_MAX) {  // bounded cache: start over once full
    SWC_HIP(hipStreamSynchronize(c->st));
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
  }
  if (!c->cap_st) SWC_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
  SWC_HIP(hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeThreadLocal));
  record(c->cap_st);
  hipGraph_t g = nullptr;
  SWC_HIP(hipStreamEndCapture(c->cap_st, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  SWC_HIP(e);
  c->graphs.push_back({key, ex});
  *out = ex;
  return SWC_OK;
}

// Steps k and k+1 can share a launch: threshold 0 (no renormalisation in
// between), a table that cannot grow during the launch, and factors with
// different XOR masks.
bool fusable(const swc_ctx* c, int64_t k, double thr, uint64_t lim) {
  return c->fuse && !c->entropy && c->tk_max == 0 && thr == 0.0 && lim == NO_LIMIT && c->hmask[k - 1] != c->hmask[k];
}

// The launches a forward range issues (issue_fwd): their number, and the
// kernel builds they use added to *builds (SWC_BUILD_* bits).
int64_t fwd_plan(const swc_ctx* c, int64_t k0, int64_t k1, double thr, uint64_t lim, int64_t* builds) {
  int64_t n = 0;
  for (int64_t k = k0; k <= k1; ++n) {
    if (k < k1 && fusable(c, k, thr, lim)) {
      *builds |= wide2(c, c->res_f2w) ? SWC_BUILD_FWD2_PRE : SWC_BUILD_FWD2;
      k += 2;
    } else {
      *builds |= c->entropy ? SWC_BUILD_FWD_ENT
                            : (hi_occ(c) ? SWC_BUILD_FWD_HO : SWC_BUILD_FWD) | (c->pf_fwd ? SWC_BUILD_FWD_PF : 0);
      n += step_launches(c) - 1;
      k += 1;
    }
  }
  return n;
}

// The same for a reverse range (issue_rev).
int64_t rev_plan(const swc_ctx* c, int64_t hi, int64_t lo, bool fuse, int64_t* builds) {
  int64_t n = 0;
  for (int64_t k = hi; k >= lo; ++n) {
    if (fuse && k > lo && c->hmask[k - 2] != c->hmask[k - 1]) {
      *builds |= wide2(c, c->res_r2w) ? SWC_BUILD_REV2_PRE : SWC_BUILD_REV2;
      k -= 2;
    } else {
      *builds |= SWC_BUILD_REV | (c->pf_rev ? SWC_BUILD_REV_PF : 0);
      n += step_launches(c) - 1;
      k -= 1;
    }
  }
  return n;
}

template <class T>
void issue_fwd(swc_ctx* c, int64_t k0, int64_t k1, double thr, int log_on, uint64_t lim, hipStream_t st) {
  for (int64_t k = k0; k <= k1;) {
    if (k < k1 && fusable(c, k, thr, lim)) {
      launch_fwd2<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, static_cast<int>(k), c->B, c->grid,
                     wide2(c, c->res_f2w), st);
      k += 2;
    } else {
      launch_fwd<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, c->lg, static_cast<int>(k), thr, k == 1,
                    log_on, lim, c->B, fwd_grid(c), split_members(c), hi_occ(c), fwd_pf(c), st);
      if (c->tk_max)
        launch_topk<T>(c->tab, c->sa, c->cnt, c->tk, static_cast<int>(k), c->tk_max, c->tk_cut, c->B, c->grid, st);
      k += 1;
    }
  }
}

// Reverse steps hi..lo (the fused pairs mirror nothing of the forward: any
// two neighbouring steps with different masks can be undone together).
template <class T>
int64_t issue_rev(swc_ctx* c, int64_t hi, int64_t lo, bool fuse, hipStream_t st) {
  int64_t n = 0;
  for (int64_t k = hi; k >= lo; ++n) {
    if (fuse && k > lo && c->hmask[k - 2] != c->hmask[k - 1]) {
      launch_rev2<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, static_cast<int>(k - 1), c->B, c->grid,
                     wide2(c, c->res_r2w), st);
      k -= 2;
    } else {
      launch_rev<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, static_cast<int>(k), c->B, rev_grid(c),
                    split_members(c), rev_pf(c), st);
      k -= 1;
    }
  }
  return n;
}

// Forward steps k0..k1 on the current table: a cached graph (`graph_ok`:
// the range starts where a chunk or a checkpoint interval starts, so the same
// ranges recur call after call), else single launches (a range resumed after
// a growth, or every launch timed).
int run_fwd_steps(swc_ctx* c, int64_t k0, int64_t k1, double thr, int log_on, uint64_t lim, bool graph_ok) {
  return dispatch(c, [&](auto* tp) -> int {
    using T = std::remove_pointer_t<decltype(tp)>;
    c->pf_fwd = c->pf_now && (c->tab.H >= PF_FWD_H || c->pf_override == 2);
    if (c->pf_fwd)
      pf_ensure<T>(c);
    else
      c->pf_valid = false;  // this range's new keys do not enter the filter
    if (c->use_graph && !c->ktiming && graph_ok) {
      const GraphKey key{0, k0, k1, thr, log_on, c->tab.H, lim, c->entropy ? 1 : 0, c->tk_max, c->tk_cut,
                         c->live ? 1 : 0, c->pf_fwd ? 1 : 0};
      hipGraphExec_t ex = nullptr;
      const int rr = cached_graph(c, key, &ex, [&](hipStream_t cs) { issue_fwd<T>(c, k0, k1, thr, log_on, lim, cs); });
      if (rr) return rr;
      SWC_HIP(hipGraphLaunch(ex, c->st));
      c->fwd_launches += fwd_plan(c, k0, k1, thr, lim, &c->builds);
      return SWC_OK;
    }
    if (!c->ktiming) {
      issue_fwd<T>(c, k0, k1, thr, log_on, lim, c->st);
      c->fwd_launches += fwd_plan(c, k0, k1, thr, lim, &c->builds);
      return SWC_OK;
    }
    c->builds |= c->entropy ? SWC_BUILD_FWD_ENT
                            : (hi_occ(c) ? SWC_BUILD_FWD_HO : SWC_BUILD_FWD) | (c->pf_fwd ? SWC_BUILD_FWD_PF : 0);
    for (int64_t k = k0; k <= k1; ++k) {  // every launch timed: one step per launch
      (void)hipEventRecord(c->kev[2 * (k - 1)], c->st);
      launch_fwd<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, c->lg, static_cast<int>(k), thr, k == 1,
                    log_on, lim, c->B, fwd_grid(c), split_members(c), hi_occ(c), fwd_pf(c), c->st);
      (void)hipEventRecord(c->kev[2 * (k - 1) + 1], c->st);
      if (c->tk_max)
        launch_topk<T>(c->tab, c->sa, c->cnt, c->tk, static_cast<int>(k), c->tk_max, c->tk_cut, c->B, c->grid,
                       c->st);
    }
    c->fwd_launches += (k1 - k0 + 1) * step_launches(c);
    return SWC_OK;
  });
}

// Checkpoint j (0-based) holds the state after forward step (j+1)*interval;
// -1 when no checkpoint is taken after step `k` of an M-step sweep.
int64_t ckpt_index(const swc_ctx* c, int64_t k, int64_t M) {
  const int64_t K = c->ck_interval;
  if (K <= 0 || k <= 0 || k >= M || k % K) return -1;
  const int64_t j = k / K - 1;
  return j < c->ck_n ? j : -1;
}

Snap ckpt_snap(const swc_ctx* c, int64_t j) {
  const size_t tsz = c->prec == SWC_FP32 ? 4 : 8;
  const size_t per = static_cast<size_t>(c->B) * c->ck_cap;
  return Snap{c->ck_key + j * per, c->ck_amp + j * per * tsz, c->ck_count + j * c->B, c->ck_cap};
}

// Last step of the range of forward steps that starts at k: the end of k's
// chunk, cut at M and, in a gradient sweep, at the next checkpoint.  A table
// that can no longer grow needs no look between the power-of-two chunks
// (wide): its ranges end only at multiples of GRAPH_CHUNK, so a short circuit
// is one graph.
int64_t fwd_range_end(const swc_ctx* c, int64_t k, int64_t M, int log_on, bool wide = false) {
  int64_t e = std::min(M, wide ? (k - 1) / GRAPH_CHUNK * GRAPH_CHUNK + GRAPH_CHUNK : chunk_end(k));
  if (log_on && c->ck_interval > 0) {
    const int64_t nxt = (k + c->ck_interval - 1) / c->ck_interval * c->ck_interval;
    if (ckpt_index(c, nxt, M) >= 0) e = std::min(e, nxt);
  }
  return e;
}

int take_checkpoint(swc_ctx* c, int64_t k, int64_t M, int log_on) {
  if (!log_on) return SWC_OK;
  const int64_t j = ckpt_index(c, k, M);
  if (j < 0) return SWC_OK;
  dispatch(c, [&](auto* tp) -> int {
    launch_snapshot<std::remove_pointer_t<decltype(tp)>>(c->tab, c->sa, ckpt_snap(c, j), static_cast<int>(k), c->B,
                                                         c->grid, c->st);
    return SWC_OK;
  });
  ++c->ck_taken;
  SWC_HIP(hipGetLastError());
  return SWC_OK;
}

// SWC_PROGRESS: wait for the work issued so far and report `done` of `total` steps
int report_progress(swc_ctx* c, const char* what, int64_t done, int64_t total) {
  if (!c->progress) return SWC_OK;
  SWC_HIP(hipStreamSynchronize(c->st));
  std::fprintf(stderr, "[swc] %s sweep: %lld of %lld steps done\n", what, static_cast<long long>(done),
               static_cast<long long>(total));
  std::fflush(stderr);
  return SWC_OK;
}

uint64_t max_occupancy(const swc_ctx* c) {
  uint64_t o = 0;
  for (int b = 0; b < c->B; ++b) o = std::max<uint64_t>(o, counter_total(c->hcnt[b], C_OCC));
  return o;
}

// The forward sweep (Eq. 3): steps 1..M in order.  While the index can still
// grow, the host reads the counters after every range of steps and rebuilds
// the index larger when the entries approach the growth limit, or when a
// step stopped the sweep at that limit (the stopped steps then run again on
// the larger index).
int forward_sweep(swc_ctx* c, int64_t M, double thr, int log_on) {
  if (c->ktiming) {
    int r0 = ensure_kev(c, static_cast<size_t>(2 * M + 2));
    if (r0) return r0;
  }
  c->rehashes = 0;
  c->compactions = 0;
  c->builds = 0;
  // the presence filter for this call's sweeps: not with persistent sweeps,
  // entropy tracking or two-factor launches (threshold 0), whose kernels
  // neither read nor keep it
  c->pf_now = !c->persistent && !c->entropy && !(thr == 0.0 && c->fuse) &&
              (c->pf_override >= 0 ? c->pf_override > 0 : c->pf_auto);
  c->sa.ea = c->entropy ? c->ent_ea : nullptr;
  c->sa.eb = c->entropy ? c->ent_eb : nullptr;
  c->ent_M = -1;
  c->live_M = -1;
  c->sa.pvis = c->live ? c->live_pvis : nullptr;
  {
    // Dead entries of earlier sweeps are dropped when they are over a quarter
    // of the entries.  The counters are current: they were read after the
    // call that left this state.
    uint64_t live = 0;
    bool compact = false;
    for (int b = 0; b < c->B; ++b) {
      const uint64_t lb = counter_total(c->hcnt[b], C_LIVE), ob = counter_total(c->hcnt[b], C_OCC);
      live = std::max(live, lb);
      compact = compact || (ob >= 1024 && 4 * (ob - std::min(ob, lb)) > ob);
    }
    if (M > 0 && compact) {
      if (int r = compact_state(c, live)) return r;
      ++c->compactions;
    }
  }
  // steps that do not use the filter do not keep it either
  if (M > 0 && !c->pf_now) c->pf_valid = false;
  dispatch(c, [&](auto* tp) -> int {
    launch_sweep_begin<std::remove_pointer_t<decltype(tp)>>(c->tab, c->sa, c->cnt, M, c->B, c->grid, c->st);
    return SWC_OK;
  });
  c->last_M = M;
  SWC_HIP(hipEventRecord(c->ev[0], c->st));
  if (c->entropy) {  // entropy of the state the sweep starts from
    dispatch(c, [&](auto* tp) -> int {
      launch_entropy_scan<std::remove_pointer_t<decltype(tp)>>(c->tab, c->sa, 0, c->B, c->grid, c->st);
      return SWC_OK;
    });
  }
  c->ck_taken = 0;
  if (log_on && c->ck_n > 0) launch_zero_u64(c->ck_count, static_cast<uint64_t>(c->ck_n) * c->B, c->st);
  c->fwd_launches = 0;
  if (c->persistent && c->tk_max == 0) {
    // one cooperative launch per range between checkpoints (the N_MAX / N_CUT
    // selection needs launches of its own after every step: per-step path)
    for (int64_t k = 1; k <= M;) {
      int64_t k1 = M;
      if (log_on && c->ck_interval > 0) {
        const int64_t nxt = (k + c->ck_interval - 1) / c->ck_interval * c->ck_interval;
        if (ckpt_index(c, nxt, M) >= 0) k1 = nxt;
      }
      launch_sync_reset(c->sy, k == 1, c->st);
      c->builds |= SWC_BUILD_PERSISTENT;
      const int r = dispatch(c, [&](auto* tp) -> int {
        using T = std::remove_pointer_t<decltype(tp)>;
        const int64_t i = c->fwd_launches;
        if (c->ktiming) (void)hipEventRecord(c->kev[2 * i], c->st);
        SWC_HIP(launch_fwd_sweep<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, c->lg, static_cast<int>(k),
                                    static_cast<int>(k1), thr, k == 1, log_on, c->sy, c->B, c->grid_fwd, c->st));
        if (c->ktiming) (void)hipEventRecord(c->kev[2 * i + 1], c->st);
        return SWC_OK;
      });
      if (r) return r;
      ++c->fwd_launches;
      if (int rr = take_checkpoint(c, k1, M, log_on)) return rr;
      k = k1 + 1;
    }
  } else {
    int64_t k = 1;
    bool resumed = false;
    double prev_occ = static_cast<double>(max_occupancy(c));  // counters read before the sweep
    while (k <= M) {
      const uint64_t lim = occ_limit(c);
      const int64_t k1 = fwd_range_end(c, k, M, log_on, lim == NO_LIMIT);
      int r = run_fwd_steps(c, k, k1, thr, log_on, lim, !resumed);
      if (r) return r;
      if (lim == NO_LIMIT) {
        if ((r = take_checkpoint(c, k1, M, log_on))) return r;
        if ((r = report_progress(c, "forward", k1, M))) return r;
        resumed = false;
        k = k1 + 1;
        continue;
      }
      launch_sweep_end(c->tab, c->sa, c->cnt, k1, k1, c->B, nullptr, 1, c->st);
      if ((r = read_counters(c))) return r;
      // a step that stopped the sweep (stop = first step not run) asks for a growth
      const uint32_t stop = c->hcnt[0].stop;
      const bool stopped = stop != ~0u;
      const int64_t next = stopped ? std::min<int64_t>(static_cast<int64_t>(stop), k1 + 1) : k1 + 1;
      bool full = false;
      for (int b = 0; b < c->B; ++b) full = full || (c->hcnt[b].flags & F_TABLE_FULL);
      if (full) break;  // reported by the caller's status check
      if (next == k1 + 1 && (r = take_checkpoint(c, k1, M, log_on))) return r;
      if ((r = report_progress(c, "forward", next - 1, M))) return r;
      const double occ = static_cast<double>(max_occupancy(c));
      const int64_t done = next - k;
      // occupancy expected at the end of the next range: the last range's
      // growth per step, extrapolated linearly with a factor-2 margin (a
      // growth that outruns it is caught by the stop)
      double pred = occ;
      if (next <= M && prev_occ >= 0.0 && done > 0) {
        const int64_t nlen = fwd_range_end(c, next, M, log_on) - next + 1;
        pred = occ + 2.0 * std::max(0.0, occ - prev_occ) * static_cast<double>(nlen) / static_cast<double>(done);
      }
      if (stopped) pred = std::max(pred, 2.0 * occ);
      if (stopped || pred > static_cast<double>(lim)) {
        if ((r = grow_table(c, static_cast<uint64_t>(std::min(pred, 1e18))))) return r;
      }
      prev_occ = occ;
      resumed = next != k1 + 1;
      k = next;
    }
  }
  launch_sweep_end(c->tab, c->sa, c->cnt, M, M, c->B, (c->persistent && M > 0) ? c->sy : nullptr, 0, c->st);
  SWC_HIP(hipEventRecord(c->ev[1], c->st));
  if (c->entropy) {
    launch_entropy_final(c->sa, M, c->B, c->st);
    c->ent_M = M;
  }
  if (c->live) c->live_M = M;
  SWC_HIP(hipGetLastError());
  return SWC_OK;
}

// The adjoint sweep, steps M..1, in ranges that end where a chunk or a
// checkpoint interval ends; after the range that reconstructs the state of a
// checkpoint, the checkpoint's amplitudes are written back over it.
// maxn[k]: largest number of truncation-log records of step k over the batch.
int reverse_sweep(swc_ctx* c, int64_t M, double thr, const std::vector<uint32_t>& maxn) {
  c->rev_launches = 0;
  // the reverse creates no keys: a filter made current once serves it all
  c->pf_rev = c->pf_now && M > 0;
  if (c->pf_rev) pf_ensure_any(c);
  c->rev_fused = c->fuse && thr == 0.0 && !c->persistent && !c->ktiming && c->log_records == 0;
  // Each step scans only the entries that existed after it in the forward
  // sweep, so the scans shrink as the sweep goes back without any rebuild;
  // ranges stop at multiples of GRAPH_CHUNK and at checkpoints.
  for (int64_t hi = M; hi >= 1;) {
    int64_t lo = (hi - 1) / GRAPH_CHUNK * GRAPH_CHUNK + 1;
    if (c->ck_interval > 0) lo = std::max(lo, (hi - 1) / c->ck_interval * c->ck_interval + 1);
    const int r = dispatch(c, [&](auto* tp) -> int {
      using T = std::remove_pointer_t<decltype(tp)>;
      if (c->persistent) {
        c->builds |= SWC_BUILD_PERSISTENT;
        launch_sync_reset(c->sy, hi == M, c->st);
        const int64_t i = c->rev_launches++;
        if (c->ktiming) (void)hipEventRecord(c->kev[2 * i], c->st);
        SWC_HIP(launch_rev_sweep<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, c->lg, static_cast<int>(hi),
                                    static_cast<int>(lo), c->sy, c->B, c->grid_rev, c->st));
        if (c->ktiming) (void)hipEventRecord(c->kev[2 * i + 1], c->st);
        return SWC_OK;
      }
      if (!c->ktiming && c->log_records == 0) {
        // no log restores interleaved: one or two steps per launch, from a
        // cached graph of the range
        const bool fz = c->fuse && thr == 0.0;
        c->rev_launches += rev_plan(c, hi, lo, fz, &c->builds);
        if (!c->use_graph) {
          issue_rev<T>(c, hi, lo, fz, c->st);
          return SWC_OK;
        }
        const GraphKey key{1, lo, hi, fz ? 0.0 : 1.0, 0, c->tab.H, 0, 0, 0, 0, 0, c->pf_rev ? 1 : 0};
        hipGraphExec_t ex = nullptr;
        const int rr = cached_graph(c, key, &ex, [&](hipStream_t cs) { issue_rev<T>(c, hi, lo, fz, cs); });
        if (rr) return rr;
        SWC_HIP(hipGraphLaunch(ex, c->st));
        return SWC_OK;
      }
      c->builds |= SWC_BUILD_REV | (c->pf_rev ? SWC_BUILD_REV_PF : 0);
      for (int64_t k = hi; k >= lo; --k) {
        if (c->ktiming) (void)hipEventRecord(c->kev[2 * (k - 1)], c->st);
        launch_rev<T>(c->tab, c->fac, c->trig, c->Mmax + 1, c->sa, c->cnt, static_cast<int>(k), c->B, rev_grid(c),
                      split_members(c), rev_pf(c), c->st);
        if (c->ktiming) (void)hipEventRecord(c->kev[2 * (k - 1) + 1], c->st);
        if (maxn[k]) launch_log_restore<T>(c->tab, c->lg, c->sa, static_cast<int>(k), c->B, maxn[k], c->st);
      }
      c->rev_launches += (hi - lo + 1) * step_launches(c);
      return SWC_OK;
    });
    if (r) return r;
    if (int rr = report_progress(c, "reverse", M - lo + 1, M)) return rr;
    const int64_t j = ckpt_index(c, lo - 1, M);
    if (j >= 0) {
      dispatch(c, [&](auto* tp) -> int {
        launch_snap_restore<std::remove_pointer_t<decltype(tp)>>(c->tab, ckpt_snap(c, j), c->cnt, c->ck_nmax[j], c->B,
                                                                 c->st);
        return SWC_OK;
      });
    }
    hi = lo - 1;
  }
  SWC_HIP(hipGetLastError());
  return SWC_OK;
}

int sweep_status(swc_ctx* c) {
  {
    uint64_t pairs = 0, hits = 0;
    for (int b = 0; b < c->B; ++b) {
      pairs += counter_total(c->hcnt[b], C_PAIRS);
      hits += counter_total(c->hcnt[b], C_HITS);
    }
    if (pairs > 0) c->pf_auto = hits <= pairs / 4;
  }
  for (int b = 0; b < c->B; ++b) {
    const Counters& k = c->hcnt[b];
    if (k.flags & F_TABLE_FULL) return fail(SWC_ECAPACITY, "hash table full");
    if (counter_total(k, C_OCC) > c->tab.H - c->tab.H / 10)
      return fail(SWC_ECAPACITY, "hash table above 90% occupancy");
    if (counter_total(k, C_LIVE) == 0) return fail(SWC_EEMPTY, "truncation removed every determinant");
    if (k.flags & F_INCONSISTENT) return fail(SWC_EDEVICE, "inconsistent pair state in the reverse sweep");
    if (k.flags & F_TIMEOUT) return fail(SWC_EDEVICE, "grid barrier of a persistent sweep timed out");
  }
  return SWC_OK;
}

// Pairing scratch: six record arrays, the radix histogram and scan sums, a
// counter and the per-determinant accumulators (one member at a time).
struct PairScratch {
  uint64_t *k0, *k1, *rI;
  uint32_t *v0, *v1, *hist, *sums;
  double* rc;
  unsigned long long* count;
  Fx3* acc;
  uint64_t cap;  // records per partition
};

bool pair_scratch(const swc_ctx* c, uint64_t nacc, PairScratch* ps) {
  if (!c->sig_buf) return false;
  const size_t fixed = align_up(sizeof(Fx3) * nacc) + align_up(4 * 4096) + align_up(8) + 16 * ALIGN;
  if (c->sig_bytes <= fixed) return false;
  uint64_t cap = static_cast<uint64_t>((c->sig_bytes - fixed) / 41);  // 40 B per record + histogram share
  cap = std::min<uint64_t>(cap, (1ull << 28) - RS_CAP_SLACK);
  if (cap < 4096) return false;
  char* p = c->sig_buf;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align_up(bytes);
    return q;
  };
  ps->k0 = reinterpret_cast<uint64_t*>(take(8 * cap));
  ps->k1 = reinterpret_cast<uint64_t*>(take(8 * cap));
  ps->rI = reinterpret_cast<uint64_t*>(take(8 * cap));
  ps->rc = reinterpret_cast<double*>(take(8 * cap));
  ps->v0 = reinterpret_cast<uint32_t*>(take(4 * cap));
  ps->v1 = reinterpret_cast<uint32_t*>(take(4 * cap));
  ps->hist = reinterpret_cast<uint32_t*>(take(4 * 256 * ((cap + 4095) / 4096)));
  ps->sums = reinterpret_cast<uint32_t*>(take(4 * 4096));
  ps->count = reinterpret_cast<unsigned long long*>(take(8));
  ps->acc = reinterpret_cast<Fx3*>(take(sizeof(Fx3) * nacc));
  ps->cap = cap;
  return static_cast<size_t>(p - c->sig_buf) <= c->sig_bytes;
}

int electrons(const swc_ctx* c) { return c->na + c->nb; }

bool use_pairs(const swc_ctx* c, int64_t nmax) {
  if (c->sig_mode == 2) return false;
  PairScratch ps;
  if (!pair_scratch(c, static_cast<uint64_t>(nmax), &ps)) return false;
  if (c->sig_mode == 1) return true;
  const uint64_t P = static_cast<uint64_t>(electrons(c)) * (electrons(c) - 1) / 2;
  return static_cast<uint64_t>(nmax) * P >= (1ull << 22);
}

// The off-diagonal part of sigma by pairing, member by member: the doubles
// from the groups of two-electron-removed keys, then the singles from the
// groups of one-electron-removed keys, partition by partition, all summed
// exactly into one accumulator per determinant.
int pair_sigma(swc_ctx* c, const double* h1, const double* h2, int64_t nmax) {
  PairScratch ps;
  if (!pair_scratch(c, static_cast<uint64_t>(nmax), &ps)) return fail(SWC_EINVAL, "sigma scratch too small");
  const uint64_t Ne = static_cast<uint64_t>(electrons(c));
  const uint64_t P[2] = {Ne * (Ne - 1) / 2, Ne};  // records per determinant: order 2, order 1
  const uint64_t H = c->cp.cs;  // stride of the compact arrays
  for (int b = 0; b < c->B; ++b) {
    const uint64_t N = c->hcnt[b].ncompact;
    if (N == 0) continue;
    int nparts[2];
    for (int o = 0; o < 2; ++o)
      nparts[o] = static_cast<int>(std::max<uint64_t>(1, (N * P[o] + N * P[o] / 4 + ps.cap - 1) / ps.cap));
    for (int attempt = 0;; ++attempt) {
      launch_fx3_zero(ps.acc, N, c->st);
      int overflow = -1;
      for (int o = 0; o < 2 && overflow < 0; ++o) {
        const int order = 2 - o;
        for (int part = 0; part < nparts[o]; ++part) {
          launch_zero_u64(ps.count, 1, c->st);
          launch_pair_emit(c->cp, H, b, N, part, nparts[o], ps.k0, ps.v0, ps.count, ps.cap, order, c->st);
          unsigned long long n = 0;
          SWC_HIP(hipMemcpyAsync(&n, ps.count, 8, hipMemcpyDeviceToHost, c->st));
          SWC_HIP(hipStreamSynchronize(c->st));
          if (n > ps.cap) {
            overflow = o;
            break;
          }
          const int flip = launch_radix_sort(ps.k0, ps.v0, ps.k1, ps.v1, n, c->nq, ps.hist, ps.sums, c->st);
          launch_pair_groups(c->cp, H, b, flip ? ps.k1 : ps.k0, flip ? ps.v1 : ps.v0, n, ps.rI, ps.rc, h1, h2,
                             c->nq / 2, ps.acc, order, c->st);
        }
      }
      if (overflow < 0) break;
      if (attempt >= 8) return fail(SWC_ECAPACITY, "sigma scratch: a partition exceeds the scratch");
      nparts[overflow] *= 2;  // an unlucky partition: split finer and start the member again
    }
    c->sig_parts = std::max<int64_t>(c->sig_parts, nparts[0]);
    launch_pair_finish(c->cp, H, b, N, ps.acc, c->st);
  }
  SWC_HIP(hipGetLastError());
  return SWC_OK;
}

// compact + sigma + E (+ lambda); leaves counters read back
// Energy, part 1: compact the live entries (their counts land in the counters).
int energy_compact(swc_ctx* c) {
  launch_energy_begin(c->cnt, c->B, c->st);
  SWC_HIP(hipEventRecord(c->ev[2], c->st));
  int r = dispatch(c, [&](auto* tp) -> int {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_compact<T>(c->tab, c->cp, c->cnt, c->B, c->grid, c->st);
    return SWC_OK;
  });
  if (r) return r;
  SWC_HIP(hipGetLastError());
  return SWC_OK;
}

// Energy, part 2 (the compact counts read into hcnt): sigma, E and, for the
// gradient, lambda_M.  Nothing here waits for the device.
int energy_run(swc_ctx* c, const double* h1, const double* h2, double* E, bool want_lambda) {
  int r = SWC_OK;
  int64_t nmax = 0;
  for (int b = 0; b < c->B; ++b) nmax = std::max<int64_t>(nmax, static_cast<int64_t>(c->hcnt[b].ncompact));
  if (nmax == 0) return fail(SWC_EEMPTY, "empty state");
  const int n = c->nq / 2;
  SWC_HIP(hipEventRecord(c->ev[6], c->st));
  const bool pairs = use_pairs(c, nmax);
  c->sig_parts = 0;
  if (pairs) {  // every off-diagonal term by pairing
    if ((r = pair_sigma(c, h1, h2, nmax))) return r;
  } else {  // every off-diagonal term by enumeration and index probes
    r = dispatch(c, [&](auto* tp) -> int {
      using T = std::remove_pointer_t<decltype(tp)>;
      launch_sigma<T>(c->tab, c->cp, c->cnt, h1, h2, c->nq, nmax, c->B, 0, c->st);
      return SWC_OK;
    });
    if (r) return r;
  }
  SWC_HIP(hipEventRecord(c->ev[7], c->st));
  launch_energy_reduce(c->cp, c->cnt, h1, h2, n, nmax, c->B, c->st);
  launch_energy_final(c->cnt, E, c->B, c->st);
  if (want_lambda) {
    r = dispatch(c, [&](auto* tp) -> int {
      using T = std::remove_pointer_t<decltype(tp)>;
      launch_lambda<T>(c->tab, c->cp, c->cnt, nmax, c->B, c->st);
      return SWC_OK;
    });
    if (r) return r;
  }
  SWC_HIP(hipEventRecord(c->ev[3], c->st));
  SWC_HIP(hipGetLastError());
  return SWC_OK;
}

int energy_impl(swc_ctx* c, const double* h1, const double* h2, double* E, bool want_lambda) {
  if (!h1 || !h2) return fail(SWC_EINVAL, "null integrals");
  int r = energy_compact(c);
  if (r || (r = read_counters(c)) || (r = energy_run(c, h1, h2, E, want_lambda))) return r;
  return read_counters(c);
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
  return ms;
}

}  // namespace

extern "C" {

size_t swc_workspace_bytes(int n_qubits, uint64_t capacity, int prec, int batch, int64_t max_factors,
                           uint64_t log_capacity) {
  if (n_qubits < 2 || n_qubits > 64 || !pow2(capacity) || capacity < 64 || capacity > (1ull << 31)) return 0;
  if ((prec != SWC_FP32 && prec != SWC_FP64) || batch < 1 || batch > 1024 || max_factors < 0 ||
      max_factors > (1ll << 30))
    return 0;
  const uint64_t L = log_capacity ? log_capacity : capacity;
  if (L > (1ull << 32)) return 0;
  return make_layout(capacity, prec == SWC_FP32 ? 4 : 8, batch, max_factors, L).total;
}

int swc_create(swc_ctx** out, int n_qubits, int n_alpha, int n_beta, uint64_t capacity, int prec, int batch,
               int64_t max_factors, uint64_t log_capacity, void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return fail(SWC_EINVAL, "null output pointer");
  *out = nullptr;
  const size_t need = swc_workspace_bytes(n_qubits, capacity, prec, batch, max_factors, log_capacity);
  if (!need) return fail(SWC_EINVAL, "invalid sizes");
  if (n_alpha < 0 || n_beta < 0 || n_alpha > n_qubits / 2 || n_beta > n_qubits / 2 ||
      n_alpha + n_beta >= n_qubits || n_alpha + n_beta == 0)
    return fail(SWC_EINVAL, "invalid electron counts");
  if (!workspace || ws_bytes < need) return fail(SWC_EINVAL, "workspace missing or too small");
  if (reinterpret_cast<uintptr_t>(workspace) % ALIGN) return fail(SWC_EINVAL, "workspace not 256-byte aligned");
  swc_ctx* c = new swc_ctx();
  c->nq = n_qubits;
  c->na = n_alpha;
  c->nb = n_beta;
  c->prec = prec;
  c->B = batch;
  c->H = capacity;
  c->Mmax = max_factors;
  c->L = log_capacity ? log_capacity : capacity;
  c->st = static_cast<hipStream_t>(stream);
  c->ws = static_cast<char*>(workspace);
  const int tsz = prec == SWC_FP32 ? 4 : 8;
  c->lay = make_layout(c->H, tsz, c->B, c->Mmax, c->L);
  const Layout& l = c->lay;
  char* w = c->ws;
  const uint64_t A = arena_size(c->H);
  c->tab = Tab{w + l.ent, w + l.aux, reinterpret_cast<Idx*>(w + l.idx), reinterpret_cast<uint32_t*>(w + l.ac), c->H,
               c->H, A};
  c->pf.w = reinterpret_cast<uint64_t*>(w + l.pf);
  c->pf.stride = c->H / 8;
  c->lg = LogArr{reinterpret_cast<uint64_t*>(w + l.lkey), reinterpret_cast<uint32_t*>(w + l.lmeta),
                 reinterpret_cast<uint32_t*>(w + l.lborn), w + l.lamp, c->L};
  c->sa = StepArr{reinterpret_cast<double*>(w + l.scale),   reinterpret_cast<Fx3*>(w + l.pw),
                  reinterpret_cast<uint32_t*>(w + l.pcnt),  reinterpret_cast<Fx3*>(w + l.gacc),
                  reinterpret_cast<uint32_t*>(w + l.logn),  reinterpret_cast<uint32_t*>(w + l.logoff),
                  reinterpret_cast<uint32_t*>(w + l.rmax),
                  reinterpret_cast<unsigned long long*>(w + l.ws),
                  static_cast<int64_t>(max_waves()),
                  c->Mmax + 1,
                  nullptr, nullptr, reinterpret_cast<double*>(w + l.entr), nullptr,
                  reinterpret_cast<uint32_t*>(w + l.nb), reinterpret_cast<uint32_t*>(w + l.app),
                  c->Mmax + 3};
  c->live_pvis = reinterpret_cast<uint32_t*>(w + l.pvis);
  c->ent_ea = reinterpret_cast<Fx3*>(w + l.ea);
  c->ent_eb = reinterpret_cast<Fx3*>(w + l.eb);
  c->cp = Compact{reinterpret_cast<uint64_t*>(w + l.ckey), reinterpret_cast<double*>(w + l.camp),
                  reinterpret_cast<uint32_t*>(w + l.cslot), reinterpret_cast<double*>(w + l.csig),
                  static_cast<uint64_t>(NA) * A};
  c->cnt = reinterpret_cast<Counters*>(w + l.cnt);
  c->fac = reinterpret_cast<FacMask*>(w + l.fac);
  c->trig = reinterpret_cast<Trig*>(w + l.trig);
  c->init_d = reinterpret_cast<uint64_t*>(w + l.init_d);
  c->init_a = reinterpret_cast<double*>(w + l.init_a);
  c->hcnt.assign(static_cast<size_t>(batch), Counters{});
  if (const char* e = std::getenv("SWC_GRID")) c->grid_override = std::max(0, std::atoi(e));  // tuning override
  if (const char* e = std::getenv("SWC_SPLIT")) c->split_override = std::atoi(e) != 0 ? 1 : 0;  // testing, tuning
  if (const char* e = std::getenv("SWC_HIOCC")) c->hiocc_override = std::atoi(e) != 0 ? 1 : 0;  // testing, tuning
  // SWC_PFILTER (testing, tuning): 0 never, 1 always, 2 always and forward steps at every index size
  if (const char* e = std::getenv("SWC_PFILTER")) c->pf_override = std::max(0, std::min(2, std::atoi(e)));
  if (const char* e = std::getenv("SWC_TABLE_MIN")) {  // smallest table after a reset (testing and tuning)
    const long long v = std::atoll(e);
    if (v >= 64 && pow2(static_cast<uint64_t>(v))) c->table_min = static_cast<uint64_t>(v);
  }
  set_table(c, c->H);
  const int g = c->grid;
  c->sy = reinterpret_cast<Sync*>(w + l.sync);
  c->tk = reinterpret_cast<TopK*>(w + l.topk);
  if (const char* e = std::getenv("SWC_SWEEP")) c->persistent = std::strcmp(e, "persistent") == 0;
  {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      delete c;
      return fail(SWC_EDEVICE, "cannot query the device");
    }
    const int bf = prec == SWC_FP32 ? resident_blocks_per_cu<float>(0) : resident_blocks_per_cu<double>(0);
    const int br = prec == SWC_FP32 ? resident_blocks_per_cu<float>(1) : resident_blocks_per_cu<double>(1);
    // co-resident blocks shared by the batch members (grid.y = batch)
    c->grid_fwd = std::min(g, bf * ncu / batch) / NA * NA;
    c->grid_rev = std::min(g, br * ncu / batch) / NA * NA;
    if (c->grid_fwd < 1 || c->grid_rev < 1) c->persistent = false;
    // resident step blocks, shared by the batch members (grid.y = batch)
    const int sf = prec == SWC_FP32 ? resident_blocks_per_cu<float>(2) : resident_blocks_per_cu<double>(2);
    const int sr = prec == SWC_FP32 ? resident_blocks_per_cu<float>(3) : resident_blocks_per_cu<double>(3);
    c->res_fwd = std::max(1, sf * ncu / batch);
    c->res_rev = std::max(1, sr * ncu / batch);
    c->res_fwd1 = std::max(1, sf * ncu);
    c->res_rev1 = std::max(1, sr * ncu);
    const int hf = prec == SWC_FP32 ? resident_blocks_per_cu<float>(7) : resident_blocks_per_cu<double>(7);
    c->res_fwdh = std::max(1, hf * ncu / batch);
    c->res_fwdh1 = std::max(1, hf * ncu);
    c->res_f2w = (prec == SWC_FP32 ? resident_blocks_per_cu<float>(5) : resident_blocks_per_cu<double>(5)) * ncu;
    c->res_r2w = (prec == SWC_FP32 ? resident_blocks_per_cu<float>(6) : resident_blocks_per_cu<double>(6)) * ncu;
    set_table(c, c->H);  // step grids with the resident limits
  }
  if (const char* e = std::getenv("SWC_KERNEL_TIMING")) c->ktiming = std::atoi(e) != 0;
  if (const char* e = std::getenv("SWC_GRAPH")) c->use_graph = std::atoi(e) != 0;
  if (const char* e = std::getenv("SWC_PROGRESS")) c->progress = std::atoi(e) != 0;
  if (const char* e = std::getenv("SWC_FUSE")) c->fuse = std::atoi(e) != 0;
  for (auto& e : c->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      swc_destroy(c);
      return fail(SWC_EDEVICE, "hipEventCreate failed");
    }
  }
  if (hipMemsetAsync(c->cnt, 0, sizeof(Counters) * batch, c->st) != hipSuccess ||
      hipMemsetAsync(c->sy, 0, sizeof(Sync), c->st) != hipSuccess ||
      hipMemsetAsync(c->tk, 0, sizeof(TopK) * batch, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess) {
    swc_destroy(c);
    return fail(SWC_EDEVICE, "initialisation failed");
  }
  *out = c;
  return SWC_OK;
}

int swc_build_state(swc_ctx* c, const uint64_t* dets, const double* amps, int64_t n) {
  if (!c) return fail(SWC_EINVAL, "null context");
  std::vector<uint64_t> d;
  std::vector<double> a;
  if (n == 0) {
    uint64_t hf = 0;
    for (int p = 0; p < c->na; ++p) hf |= 1ull << (2 * p);
    for (int p = 0; p < c->nb; ++p) hf |= 1ull << (2 * p + 1);
    d.push_back(hf);
    a.push_back(1.0);
  } else {
    if (n < 0 || !dets || !amps) return fail(SWC_EINVAL, "invalid initial state arrays");
    if (static_cast<uint64_t>(n) > c->H / 2) return fail(SWC_EINVAL, "initial state larger than half the table");
    std::unordered_set<uint64_t> seen;
    for (int64_t i = 0; i < n; ++i) {
      if (dets[i] == EMPTY_KEY || (c->nq < 64 && (dets[i] >> c->nq)))
        return fail(SWC_EINVAL, "determinant uses bits at or above n_qubits");
      if (!std::isfinite(amps[i])) return fail(SWC_EINVAL, "non-finite amplitude");
      if (!seen.insert(dets[i]).second) return fail(SWC_EINVAL, "duplicate determinant");
    }
    d.assign(dets, dets + n);
    a.assign(amps, amps + n);
  }
  double n2 = 0.0;
  for (double v : a) n2 += v * v;
  if (!(n2 > 0.0)) return fail(SWC_EINVAL, "initial state has zero norm");
  c->h_init_d = std::move(d);
  c->h_init_a = std::move(a);
  c->S0 = 1.0 / std::sqrt(n2);
  // |Psi_0> stays on the device for every later reset
  const size_t n0 = c->h_init_d.size();
  SWC_HIP(hipMemcpyAsync(c->init_d, c->h_init_d.data(), 8 * n0, hipMemcpyHostToDevice, c->st));
  SWC_HIP(hipMemcpyAsync(c->init_a, c->h_init_a.data(), 8 * n0, hipMemcpyHostToDevice, c->st));
  int r = reset_state(c);
  if (r) return r;
  if ((r = read_counters(c))) return r;
  for (int b = 0; b < c->B; ++b)
    if (c->hcnt[b].flags & F_TABLE_FULL) return fail(SWC_ECAPACITY, "hash table full");
  c->built = true;
  return SWC_OK;
}

int swc_apply_ucc(swc_ctx* c, const double* theta, const swc_exc* exc, int64_t M, double threshold) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  if (!c->built) return fail(SWC_ESTATE, "no state built");
  if (M < 0 || M > c->Mmax) return fail(SWC_EINVAL, "factor count above max_factors");
  if (!(threshold >= 0.0) || !std::isfinite(threshold)) return fail(SWC_EINVAL, "threshold must be finite and >= 0");
  int r = check_exc(c->nq, exc, M);
  if (r) return r;
  if ((r = upload_masks(c, exc, M))) return r;
  if ((r = check_theta(c, theta, M))) return r;
  if ((r = forward_sweep(c, M, threshold, 0))) return r;
  if ((r = read_counters(c))) return r;
  c->fwd_ms = elapsed(c->ev[0], c->ev[1]);
  if (c->ktiming) {  // event pairs: one per launch (persistent) or per step
    c->rot_n = c->persistent ? c->fwd_launches : M;
    c->rot_ms = sum_pairs(c, c->rot_n);
  }
  r = sweep_status(c);
  if (r) c->built = false;
  return r;
}

int swc_energy(swc_ctx* c, const double* h1, const double* h2, double* E) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  if (!c->built) return fail(SWC_ESTATE, "no state built");
  if (!E) return fail(SWC_EINVAL, "null output");
  int r = energy_impl(c, h1, h2, E, false);
  if (r) return r;
  c->energy_ms = elapsed(c->ev[2], c->ev[3]);
  c->sig_ms = elapsed(c->ev[6], c->ev[7]);
  return SWC_OK;
}

int swc_energy_and_grad(swc_ctx* c, const double* theta, const swc_exc* exc, int64_t M, double threshold,
                        const double* h1, const double* h2, double* E, double* grad) {
  if (!c) return fail(SWC_EINVAL, "null context");
  if (!c->built) return fail(SWC_ESTATE, "no state built");
  if (M < 0 || M > c->Mmax) return fail(SWC_EINVAL, "factor count above max_factors");
  if (!(threshold >= 0.0) || !std::isfinite(threshold)) return fail(SWC_EINVAL, "threshold must be finite and >= 0");
  if (!E || (M > 0 && !grad)) return fail(SWC_EINVAL, "null output");
  if (!h1 || !h2) return fail(SWC_EINVAL, "null integrals");
  int r = check_exc(c->nq, exc, M);
  if (r) return r;
  if ((r = upload_masks(c, exc, M))) return r;
  // a call that follows a reset (the end of the previous gradient call, or
  // build_state) with nothing in between starts from that table as it is
  if (!c->fresh && (r = reset_state(c))) return r;
  c->fresh = false;
  // the angle check's flag is read with the forward sweep's status below
  if ((r = check_theta(c, theta, M, false))) return r;
  if ((r = forward_sweep(c, M, threshold, 1))) return r;
  if ((r = energy_compact(c))) return r;
  // One host wait for the sweep's status, the compact counts, the per-step
  // log sizes and the checkpoint sizes.
  const int64_t S = c->Mmax + 1;
  std::vector<uint32_t> logn(static_cast<size_t>(c->B * S)), logoff(static_cast<size_t>(c->B * S), 0u);
  std::vector<unsigned long long> cnts(static_cast<size_t>(c->ck_taken) * c->B);
  SWC_HIP(hipMemcpyAsync(c->hcnt.data(), c->cnt, sizeof(Counters) * c->B, hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipMemcpyAsync(logn.data(), c->sa.logn, 4 * c->B * S, hipMemcpyDeviceToHost, c->st));
  if (c->ck_taken > 0)
    SWC_HIP(hipMemcpyAsync(cnts.data(), c->ck_count, 8 * cnts.size(), hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipStreamSynchronize(c->st));
  if (M > 0 && (c->hcnt[0].flags & F_BAD_THETA)) {
    reset_state(c);
    return fail(SWC_EINVAL, "theta contains a non-finite value");
  }
  if ((r = sweep_status(c))) {
    reset_state(c);
    return r;
  }
  for (int b = 0; b < c->B; ++b)
    if (c->hcnt[b].flags & F_LOG_FULL) {
      const unsigned long long need = c->hcnt[b].logcnt;
      reset_state(c);
      return fail(SWC_ECAPACITY, "truncation log full: " + std::to_string(need) + " records needed, capacity " +
                                     std::to_string(c->L));
    }
  if (c->ck_taken > 0) {
    c->ck_nmax.assign(static_cast<size_t>(c->ck_n), 0);
    for (int64_t j = 0; j < c->ck_taken; ++j)
      for (int b = 0; b < c->B; ++b) c->ck_nmax[j] = std::max<uint64_t>(c->ck_nmax[j], cnts[j * c->B + b]);
    for (int64_t j = 0; j < c->ck_taken; ++j)
      if (c->ck_nmax[j] > c->ck_cap) {
        reset_state(c);
        return fail(SWC_ECAPACITY, "checkpoint holds fewer entries than the state");
      }
  }
  c->fwd_ms = elapsed(c->ev[0], c->ev[1]);
  if (c->ktiming) {  // event pairs: one per launch (persistent) or per step
    c->rot_n = c->persistent ? c->fwd_launches : M;
    c->rot_ms = sum_pairs(c, c->rot_n);
  }
  if ((r = energy_run(c, h1, h2, E, true))) {
    reset_state(c);
    return r;
  }
  // offsets of the per-step truncation-log records
  std::vector<uint32_t> maxn(static_cast<size_t>(M + 1), 0u);
  c->log_records = 0;
  for (int b = 0; b < c->B; ++b) {
    uint32_t off = 0;
    for (int64_t k = 0; k <= M; ++k) {
      logoff[b * S + k] = off;
      off += logn[b * S + k];
      maxn[k] = std::max(maxn[k], logn[b * S + k]);
    }
    c->log_records += off;
  }
  if (c->log_records) {
    SWC_HIP(hipMemcpyAsync(c->sa.logoff, logoff.data(), 4 * c->B * S, hipMemcpyHostToDevice, c->st));
  }
  if (c->persistent && M > 0) {
    SWC_HIP(hipMemcpyAsync(c->sa.rmax, maxn.data(), 4 * (M + 1), hipMemcpyHostToDevice, c->st));
  }
  SWC_HIP(hipEventRecord(c->ev[4], c->st));
  if ((r = reverse_sweep(c, M, threshold, maxn))) return r;
  launch_grad_final(c->sa, c->cnt, grad, M, c->B, c->st);
  SWC_HIP(hipEventRecord(c->ev[5], c->st));
  if (c->persistent && M > 0) launch_sweep_end(c->tab, c->sa, c->cnt, 0, 0, c->B, c->sy, 0, c->st);  // barrier status only
  SWC_HIP(hipGetLastError());
  // One host wait for the adjoint sweep's status and the counters of the
  // state it leaves (|Psi_0> again, rebuilt right away).
  std::vector<Counters> after(static_cast<size_t>(c->B));
  SWC_HIP(hipMemcpyAsync(after.data(), c->cnt, sizeof(Counters) * c->B, hipMemcpyDeviceToHost, c->st));
  if ((r = reset_state(c))) return r;
  SWC_HIP(hipMemcpyAsync(c->hcnt.data(), c->cnt, sizeof(Counters) * c->B, hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipStreamSynchronize(c->st));
  c->energy_ms = elapsed(c->ev[2], c->ev[3]);
  c->sig_ms = elapsed(c->ev[6], c->ev[7]);
  c->rev_ms = elapsed(c->ev[4], c->ev[5]);
  if (c->ktiming) {
    c->revk_n = c->persistent ? c->rev_launches : M;
    c->revk_ms = sum_pairs(c, c->revk_n);
  }
  ++c->grad_calls;
  c->fwd_ms_total += c->fwd_ms;
  c->rev_ms_total += c->rev_ms;
  c->sig_ms_total += c->sig_ms;
  for (int b = 0; b < c->B; ++b) {
    if (after[b].flags & (F_INCONSISTENT | F_TIMEOUT))
      return fail(SWC_EDEVICE, (after[b].flags & F_TIMEOUT) ? "grid barrier of a persistent sweep timed out"
                                                            : "inconsistent pair state in the reverse sweep");
    if (after[b].flags & F_TABLE_FULL)  // no reverse kernel inserts: a guard
      return fail(SWC_ECAPACITY, "hash table full in the reverse sweep");
  }
  return SWC_OK;
}

size_t swc_checkpoint_bytes(int prec, int batch, int64_t max_factors, int64_t interval, uint64_t max_entries) {
  if ((prec != SWC_FP32 && prec != SWC_FP64) || batch < 1 || max_factors < 0 || interval < 1 || max_entries < 1 ||
      max_entries > (1ull << 34))
    return 0;
  const size_t tsz = prec == SWC_FP32 ? 4 : 8;
  const size_t n = max_factors > 0 ? static_cast<size_t>((max_factors - 1) / interval) : 0;
  const size_t per = static_cast<size_t>(batch) * max_entries;
  return align_up(n * per * 8) + align_up(n * per * tsz) + align_up(n * batch * 8) + ALIGN;
}

int swc_set_checkpoints(swc_ctx* c, int64_t interval, uint64_t max_entries, void* buffer, size_t bytes) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  if (interval <= 0) {
    c->ck_interval = 0;
    c->ck_n = 0;
    c->ck_cap = 0;
    return SWC_OK;
  }
  const size_t need = swc_checkpoint_bytes(c->prec, c->B, c->Mmax, interval, max_entries);
  if (!need) return fail(SWC_EINVAL, "invalid checkpoint sizes");
  if (!buffer || bytes < need) return fail(SWC_EINVAL, "checkpoint buffer missing or too small");
  if (reinterpret_cast<uintptr_t>(buffer) % ALIGN) return fail(SWC_EINVAL, "checkpoint buffer not 256-byte aligned");
  const size_t tsz = c->prec == SWC_FP32 ? 4 : 8;
  const size_t n = c->Mmax > 0 ? static_cast<size_t>((c->Mmax - 1) / interval) : 0;
  const size_t per = static_cast<size_t>(c->B) * max_entries;
  char* p = static_cast<char*>(buffer);
  c->ck_interval = interval;
  c->ck_cap = max_entries;
  c->ck_n = static_cast<int64_t>(n);
  c->ck_key = reinterpret_cast<uint64_t*>(p);
  c->ck_amp = p + align_up(n * per * 8);
  c->ck_count = reinterpret_cast<unsigned long long*>(p + align_up(n * per * 8) + align_up(n * per * tsz));
  c->ck_nmax.assign(n, 0);
  return SWC_OK;
}

int swc_set_sigma_scratch(swc_ctx* c, void* buffer, size_t bytes, int mode) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  if (mode < 0 || mode > 2) return fail(SWC_EINVAL, "mode must be 0 (auto), 1 (always) or 2 (never)");
  if (buffer && reinterpret_cast<uintptr_t>(buffer) % ALIGN) return fail(SWC_EINVAL, "scratch not 256-byte aligned");
  c->sig_buf = static_cast<char*>(buffer);
  c->sig_bytes = buffer ? bytes : 0;
  c->sig_mode = buffer ? mode : 2;
  PairScratch ps;
  if (buffer && mode != 2 && !pair_scratch(c, 1, &ps)) return fail(SWC_EINVAL, "sigma scratch too small");
  return SWC_OK;
}

int swc_set_topk(swc_ctx* c, uint64_t n_max, uint64_t n_cut) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  if (n_max == 0 && n_cut == 0) {
    c->tk_max = c->tk_cut = 0;
    return SWC_OK;
  }
  if (n_cut < 1 || n_cut > n_max) return fail(SWC_EINVAL, "need 1 <= n_cut <= n_max");
  c->tk_max = n_max;
  c->tk_cut = n_cut;
  return SWC_OK;
}

int swc_track_entropy(swc_ctx* c, int on) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  c->entropy = on != 0;
  return SWC_OK;
}

int swc_track_live(swc_ctx* c, int on) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  c->live = on != 0;
  return SWC_OK;
}

int swc_get_entropy(swc_ctx* c, int b, double* S, int64_t n) {
  if (!c) return fail(SWC_EINVAL, "null context");
  if (c->ent_M < 0) return fail(SWC_ESTATE, "entropy was not tracked in the last forward sweep");
  if (b < 0 || b >= c->B || !S) return fail(SWC_EINVAL, "bad batch index or output");
  if (n < c->ent_M + 1) return fail(SWC_EINVAL, "output holds fewer than M + 1 values");
  SWC_HIP(hipMemcpyAsync(S, c->sa.ent + b * c->sa.stride, 8 * (c->ent_M + 1), hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipStreamSynchronize(c->st));
  return SWC_OK;
}

int swc_get_live_counts(swc_ctx* c, int b, int64_t* n, int64_t len) {
  if (!c) return fail(SWC_EINVAL, "null context");
  if (c->live_M < 0) return fail(SWC_ESTATE, "live counts were not tracked in the last forward sweep");
  if (b < 0 || b >= c->B || !n) return fail(SWC_EINVAL, "bad batch index or output");
  const int64_t M = c->live_M;
  if (len < M + 1) return fail(SWC_EINVAL, "output holds fewer than M + 1 values");
  if (M == 0) {  // no step ran: the state the sweep started from is still there
    if (int r = read_counters(c)) return r;
    n[0] = static_cast<int64_t>(counter_total(c->hcnt[b], C_LIVE));
    return SWC_OK;
  }
  // the SH shards of member b: (b*SH + sh)*stride + k, one block
  const int64_t stride = c->sa.stride;
  std::vector<uint32_t> h(static_cast<size_t>(SH * stride));
  SWC_HIP(hipMemcpyAsync(h.data(), c->live_pvis + static_cast<int64_t>(b) * SH * stride, 4 * h.size(),
                         hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipStreamSynchronize(c->st));
  for (int64_t k = 1; k <= M; ++k) {
    int64_t v = 0;
    for (int sh = 0; sh < SH; ++sh) v += h[static_cast<size_t>(sh * stride + k)];
    n[k - 1] = v;
  }
  n[M] = h[0];
  return SWC_OK;
}

int swc_get_state(swc_ctx* c, int b, uint64_t* dets, double* amps, int64_t cap, int64_t* n_out) {
  if (!c) return fail(SWC_EINVAL, "null context");
  c->fresh = false;
  if (!c->built) return fail(SWC_ESTATE, "no state built");
  if (b < 0 || b >= c->B || !n_out) return fail(SWC_EINVAL, "bad batch index or output");
  launch_energy_begin(c->cnt, c->B, c->st);
  int r = dispatch(c, [&](auto* tp) -> int {
    using T = std::remove_pointer_t<decltype(tp)>;
    launch_compact<T>(c->tab, c->cp, c->cnt, c->B, c->grid, c->st);
    return SWC_OK;
  });
  if (r) return r;
  SWC_HIP(hipGetLastError());
  if ((r = read_counters(c))) return r;
  const int64_t n = static_cast<int64_t>(c->hcnt[b].ncompact);
  *n_out = n;
  if (n > cap) return fail(SWC_ECAPACITY, "output arrays too small");
  std::vector<uint64_t> k(static_cast<size_t>(n));
  std::vector<double> a(static_cast<size_t>(n));
  SWC_HIP(hipMemcpyAsync(k.data(), c->cp.key + b * c->cp.cs, 8 * n, hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipMemcpyAsync(a.data(), c->cp.amp + b * c->cp.cs, 8 * n, hipMemcpyDeviceToHost, c->st));
  SWC_HIP(hipStreamSynchronize(c->st));
  std::vector<int64_t> idx(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return k[x] < k[y]; });
  double n2 = 0.0;
  for (int64_t i = 0; i < n; ++i) n2 += a[idx[i]] * a[idx[i]];
  const double inv = n2 > 0.0 ? 1.0 / std::sqrt(n2) : 0.0;
  for (int64_t i = 0; i < n; ++i) {
    dets[i] = k[idx[i]];
    amps[i] = a[idx[i]] * inv;
  }
  return SWC_OK;
}

int swc_get_stats(swc_ctx* c, swc_stats* out) {
  if (!c || !out) return fail(SWC_EINVAL, "null argument");
  if (c->last_M > 0) launch_scan_totals(c->sa, c->cnt, c->last_M, c->B, c->st);
  int r = read_counters(c);
  if (r) return r;
  swc_stats s{};
  for (int b = 0; b < c->B; ++b) {
    const Counters& k = c->hcnt[b];
    s.det_updates += static_cast<int64_t>(counter_total(k, C_DU));
    s.pair_updates += static_cast<int64_t>(counter_total(k, C_PAIRS));
    s.inserts += static_cast<int64_t>(counter_total(k, C_INS));
    s.pruned += static_cast<int64_t>(counter_total(k, C_PRUNED));
  }
  s.n_live = static_cast<int64_t>(counter_total(c->hcnt[0], C_LIVE));
  s.slots_used = static_cast<int64_t>(counter_total(c->hcnt[0], C_OCC));
  s.log_records = c->log_records;
  s.table_slots = static_cast<int64_t>(c->tab.H);
  s.rehashes = c->rehashes;
  s.compactions = c->compactions;
  s.shrinks = 0;
  s.kernel_builds = c->builds;
  for (int b = 0; b < c->B; ++b) {
    s.fwd_slots_scanned += static_cast<int64_t>(c->hcnt[b].sh[0].v[C_FSCAN]);
    s.rev_slots_scanned += static_cast<int64_t>(c->hcnt[b].sh[0].v[C_RSCAN]);
  }
  s.checkpoints = c->ck_taken;
  s.sigma_partitions = c->sig_parts;
  s.fwd_ms = c->fwd_ms;
  s.energy_ms = c->energy_ms;
  s.rev_ms = c->rev_ms;
  s.rotate_kernel_ms = c->rot_ms;
  s.rotate_launches = c->ktiming ? c->rot_n : c->fwd_launches;
  s.reverse_kernel_ms = c->revk_ms;
  s.reverse_launches = c->ktiming ? c->revk_n : c->rev_launches;
  s.sigma_kernel_ms = c->sig_ms;
  for (int b = 0; b < c->B; ++b) s.partner_hits += static_cast<int64_t>(counter_total(c->hcnt[b], C_HITS));
  s.grad_calls = c->grad_calls;
  s.fwd_ms_total = c->fwd_ms_total;
  s.rev_ms_total = c->rev_ms_total;
  s.sigma_kernel_ms_total = c->sig_ms_total;
  *out = s;
  return SWC_OK;
}

const char* swc_strerror(int code) {
  switch (code) {
    case SWC_OK: return "ok";
    case SWC_EINVAL: return "invalid argument";
    case SWC_ECAPACITY: return "capacity exceeded";
    case SWC_EEMPTY: return "state became empty";
    case SWC_EDEVICE: return "HIP device error";
    case SWC_ESTATE: return "no state built";
    default: return "unknown error";
  }
}

const char* swc_last_error(void) { return g_err.c_str(); }

void swc_destroy(swc_ctx* c) {
  if (!c) return;
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->kev) (void)hipEventDestroy(e);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  if (c->cap_st) (void)hipStreamDestroy(c->cap_st);
  delete c;
}

int swc_validate_excitations(int n_qubits, const swc_exc* exc, int64_t M) {
  if (n_qubits < 2 || n_qubits > 64) return fail(SWC_EINVAL, "n_qubits out of range");
  return check_exc(n_qubits, exc, M);
}

int swc_factor_masks(int n_qubits, const swc_exc* exc, int64_t M, uint64_t* masks) {
  int r = swc_validate_excitations(n_qubits, exc, M);
  if (r) return r;
  for (int64_t k = 0; k < M; ++k) {
    const FacMask f = factor_mask(exc[k]);
    masks[3 * k] = f.occ;
    masks[3 * k + 1] = f.vir;
    masks[3 * k + 2] = f.sgn;
  }
  return SWC_OK;
}

}  // extern "C"
