// HIP kernels of the sparse wavefunction circuit (gfx950).
//
// State layout (per batch member): the determinants are entries of dense
// arrays, split into NA arenas that grow by appending; an open-addressed hash
// index (linear probing on a 64-bit mixer of the determinant) maps a
// determinant to its entry id.  Entry arrays are array-of-structs, so one
// load returns key, state word and amplitude:
//   float  states: 16-byte entry {key, amp, meta} + 8-byte side entry {lam, born}
//   double states: 32-byte entry {key, amp, lam, meta, born}
// Sweep steps scan the entries (a block takes one arena), not the slots of a
// hash table; a determinant pair touched by a factor is updated by exactly one
// lane (the lower member if it is present, else the upper one), so no
// amplitude is ever written by two lanes.
//
// Cross-lane rules inside one step kernel:
//  * new entries are appended to the creating wave's arena (one returning
//    atomic per wave) and indexed with atomicCAS on an EMPTY index key, so two
//    inserts never share an entry or an index slot;
//  * the entries an arena held when the launch began are known to every lane
//    (the counts of the previous launch plus its appends), so an entry created
//    by the launch itself is recognised from its id alone, without reading it;
//  * "present at the start of step k" is read from meta as
//    alive-and-not-born-in-k, or dead-with-tag-k (killed in this step); every
//    write a lane makes during step k keeps that predicate unchanged, so a
//    partner's presence test gives the same answer whenever it runs;
//  * floating-point reductions are exact 128-bit fixed-point integer sums,
//    spread over shards in separate cache lines.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "swc_internal.h"

namespace swc {

constexpr int BLK = 256;

// ---------------------------------------------------------------------------
// state views
// ---------------------------------------------------------------------------

template <class T>
struct View;

template <>
struct View<float> {
  Slot<float>* sl;  // entries of the member
  AuxF* aux;
  Idx* ix;          // index of the member
  uint64_t H, A;
  __device__ float& lam(uint64_t e) const { return aux[e].lam; }
  __device__ uint32_t& born(uint64_t e) const { return aux[e].born; }
  __device__ float lam_of(const Slot<float>&, uint64_t e) const { return aux[e].lam; }
  // split load: issue lam_pre(e) early, combine with the entry later
  __device__ float lam_pre(uint64_t e) const { return aux[e].lam; }
  __device__ float lam_fin(const Slot<float>&, float pre) const { return pre; }
  __device__ uint64_t off(uint32_t id) const { return (id >> ID_POS_BITS) * A + (id & ID_POS_MASK); }
};

template <>
struct View<double> {
  Slot<double>* sl;
  Idx* ix;
  uint64_t H, A;
  __device__ double& lam(uint64_t e) const { return sl[e].lam; }
  __device__ uint32_t& born(uint64_t e) const { return sl[e].born; }
  __device__ double lam_of(const Slot<double>& v, uint64_t) const { return v.lam; }
  __device__ double lam_pre(uint64_t) const { return 0.0; }
  __device__ double lam_fin(const Slot<double>& v, double) const { return v.lam; }
  __device__ uint64_t off(uint32_t id) const { return (id >> ID_POS_BITS) * A + (id & ID_POS_MASK); }
};

template <class T>
__device__ __forceinline__ View<T> view(const Tab& t, int b);
template <>
__device__ __forceinline__ View<float> view<float>(const Tab& t, int b) {
  const uint64_t E = static_cast<uint64_t>(NA) * t.A;
  return View<float>{static_cast<Slot<float>*>(t.ent) + b * E, static_cast<AuxF*>(t.aux) + b * E,
                     t.idx + b * t.Hcap, t.H, t.A};
}
template <>
__device__ __forceinline__ View<double> view<double>(const Tab& t, int b) {
  const uint64_t E = static_cast<uint64_t>(NA) * t.A;
  return View<double>{static_cast<Slot<double>*>(t.ent) + b * E, t.idx + b * t.Hcap, t.H, t.A};
}

__device__ __forceinline__ uint32_t entry_id(int arena, uint64_t pos) {
  return (static_cast<uint32_t>(arena) << ID_POS_BITS) | static_cast<uint32_t>(pos);
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__device__ __forceinline__ Fx fx_zero() { return Fx{0ull, 0ull}; }

__device__ __forceinline__ Fx fx_add(Fx a, Fx b) {
  Fx r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
  return r;
}

// floor(v * 2^96) as 128-bit two's complement; |v| < 2^31.
__device__ __forceinline__ Fx fx_from(double v) {
  const double t = v * 0x1p32;
  const double h = floor(t);
  const double f = t - h;  // exact, in [0, 1)
  Fx r;
  r.hi = static_cast<unsigned long long>(static_cast<long long>(h));
  r.lo = static_cast<unsigned long long>(f * 0x1p64);
  return r;
}

__device__ __forceinline__ double fx_to_d(Fx a) {
  return static_cast<double>(static_cast<long long>(a.hi)) * 0x1p-32 + static_cast<double>(a.lo) * 0x1p-96;
}

__device__ __forceinline__ bool fx_nonzero(Fx a) { return (a.lo | a.hi) != 0ull; }

__device__ __forceinline__ void fx3_atomic_add(Fx3* dst, Fx v) {
  constexpr unsigned long long M42 = (1ull << 42) - 1ull;
  const unsigned long long l0 = v.lo & M42;
  const unsigned long long l1 = ((v.lo >> 42) | (v.hi << 22)) & M42;
  const long long l2 = static_cast<long long>(v.hi) >> 20;
  atomicAdd(&dst->l[0], l0);
  atomicAdd(&dst->l[1], l1);
  atomicAdd(&dst->l[2], static_cast<unsigned long long>(l2));
}

__device__ __forceinline__ Fx fx3_value(const Fx3& a) {
  Fx r;
  r.lo = 0ull;
  r.hi = static_cast<unsigned long long>(static_cast<long long>(a.l[2])) << 20;
  Fx t;
  t.lo = a.l[1] << 42;
  t.hi = a.l[1] >> 22;
  r = fx_add(r, t);
  t.lo = a.l[0];
  t.hi = 0ull;
  return fx_add(r, t);
}

__device__ __forceinline__ Fx3 fx3_zero() { return Fx3{{0ull, 0ull, 0ull}}; }

// Wave sums through DPP lane moves (no LDS round trips).  Six steps, each
// adding a moved copy: quad_perm [1,0,3,2] and [2,3,0,1] (quad sums),
// row_half_mirror and row_mirror (row sums, every lane of a row), row_bcast
// 15 into rows 1 and 3, row_bcast 31 into rows 2 and 3: lane 63 then holds
// the total, read back as a wave-uniform value.  Lanes of rows a step leaves
// out receive 0.  The sums are integer (exact), so the grouping does not
// matter; every lane of the wave must be active.
constexpr int DPP_QUAD_1032 = 0xb1, DPP_QUAD_2301 = 0x4e, DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141,
              DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned int dpp_u32(unsigned int v) {
  return static_cast<unsigned int>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROWS, 0xf, false));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const unsigned int lo = dpp_u32<CTRL, ROWS>(static_cast<unsigned int>(v));
  const unsigned int hi = dpp_u32<CTRL, ROWS>(static_cast<unsigned int>(v >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ unsigned long long lane63_u64(unsigned long long v) {
  const unsigned int lo = static_cast<unsigned int>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
  const unsigned int hi = static_cast<unsigned int>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), 63));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ Fx dpp_fx(Fx v) {
  return Fx{dpp_u64<CTRL, ROWS>(v.lo), dpp_u64<CTRL, ROWS>(v.hi)};
}

__device__ __forceinline__ Fx wave_fx(Fx v) {
  v = fx_add(v, dpp_fx<DPP_QUAD_1032, 0xf>(v));
  v = fx_add(v, dpp_fx<DPP_QUAD_2301, 0xf>(v));
  v = fx_add(v, dpp_fx<DPP_ROW_HALF_MIRROR, 0xf>(v));
  v = fx_add(v, dpp_fx<DPP_ROW_MIRROR, 0xf>(v));
  v = fx_add(v, dpp_fx<DPP_ROW_BCAST15, 0xa>(v));
  v = fx_add(v, dpp_fx<DPP_ROW_BCAST31, 0xc>(v));
  return Fx{lane63_u64(v.lo), lane63_u64(v.hi)};
}

__device__ __forceinline__ unsigned int wave_u32(unsigned int v) {
  v += dpp_u32<DPP_QUAD_1032, 0xf>(v);
  v += dpp_u32<DPP_QUAD_2301, 0xf>(v);
  v += dpp_u32<DPP_ROW_HALF_MIRROR, 0xf>(v);
  v += dpp_u32<DPP_ROW_MIRROR, 0xf>(v);
  v += dpp_u32<DPP_ROW_BCAST15, 0xa>(v);
  v += dpp_u32<DPP_ROW_BCAST31, 0xc>(v);
  return static_cast<unsigned int>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

__device__ __forceinline__ unsigned long long wave_u64(unsigned long long v) {
  v += dpp_u64<DPP_QUAD_1032, 0xf>(v);
  v += dpp_u64<DPP_QUAD_2301, 0xf>(v);
  v += dpp_u64<DPP_ROW_HALF_MIRROR, 0xf>(v);
  v += dpp_u64<DPP_ROW_MIRROR, 0xf>(v);
  v += dpp_u64<DPP_ROW_BCAST15, 0xa>(v);
  v += dpp_u64<DPP_ROW_BCAST31, 0xc>(v);
  return lane63_u64(v);
}

// block-wide sums of one Fx and up to 7 counters (32-bit: per-launch counts
// of one state stay below 2^32); result valid in thread 0
struct Red {
  Fx f;
  unsigned int c[7];
};

__device__ __forceinline__ Red block_reduce(Red r) {
  __shared__ Red part[BLK / 64];
  r.f = wave_fx(r.f);
#pragma unroll
  for (int i = 0; i < 7; ++i) r.c[i] = wave_u32(r.c[i]);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) part[w] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < static_cast<int>(blockDim.x >> 6); ++i) {
      r.f = fx_add(r.f, part[i].f);
#pragma unroll
      for (int j = 0; j < 7; ++j) r.c[j] += part[i].c[j];
    }
  }
  return r;
}


// ---------------------------------------------------------------------------
// index probes
// ---------------------------------------------------------------------------

// Linear probe for `key`; on a hit returns the index slot and its contents
// (one whole-slot load per probe step), else -1 and the first EMPTY slot seen.
// The linear probe for `key` starts at the first slot of its 4-slot group
// (64 bytes, one aligned memory segment), so the first load of a probe brings
// in the whole group: with the index at most 45% full, nearly every probe
// ends inside it.  (H is a power of two >= 64.)
__device__ __forceinline__ uint64_t home_slot(uint64_t key, uint64_t H) { return mix64(key) & (H - 1) & ~3ull; }

__device__ __forceinline__ int64_t find_slot(const Idx* __restrict__ ix, uint64_t H, uint64_t key,
                                             uint64_t* first_free, Idx* out) {
  const uint64_t mask = H - 1;
  uint64_t s = home_slot(key, H);
  for (uint64_t i = 0; i < H; ++i, s = (s + 1) & mask) {
    const Idx v = ix[s];
    if (v.key == key) {
      *out = v;
      return static_cast<int64_t>(s);
    }
    if (v.key == EMPTY_KEY) {
      *first_free = s;
      return -1;
    }
  }
  *first_free = H;
  return -1;
}

// find_slot with the home slot already loaded (`v` = ix[home]), so several
// probes can have their first loads in flight together.  Past the home slot
// the probe loads PG slots at a time and checks them in order (the same
// answer as one slot at a time: the loads are only issued together), so a
// long probe sequence costs one round trip per PG slots rather than per slot.
constexpr int PG = 4;
// slots from the home loaded up front by the two-factor sweep kernels when
// one launch covers the state in one pass
constexpr int PH2 = 4;

__device__ __forceinline__ int64_t probe_past(const Idx* __restrict__ ix, uint64_t H, uint64_t key, uint64_t s,
                                              uint64_t i0, uint64_t* first_free, Idx* out) {
  const uint64_t mask = H - 1;
  for (uint64_t i = i0; i < H; i += PG) {
    Idx w[PG];
#pragma unroll
    for (int j = 0; j < PG; ++j) w[j] = ix[(s + 1 + j) & mask];
#pragma unroll
    for (int j = 0; j < PG; ++j) {
      const uint64_t t = (s + 1 + j) & mask;
      if (w[j].key == key) {
        *out = w[j];
        return static_cast<int64_t>(t);
      }
      if (w[j].key == EMPTY_KEY) {
        *first_free = t;
        return -1;
      }
    }
    s = (s + PG) & mask;
  }
  *first_free = H;
  return -1;
}

__device__ __forceinline__ int64_t find_slot_from(const Idx* __restrict__ ix, uint64_t H, uint64_t key, uint64_t home,
                                                  Idx v, uint64_t* first_free, Idx* out) {
  if (v.key == key) {
    *out = v;
    return static_cast<int64_t>(home);
  }
  if (v.key == EMPTY_KEY) {
    *first_free = home;
    return -1;
  }
  return probe_past(ix, H, key, home, 1, first_free, out);
}

// find_slot_from with the first PH slots from home already loaded
// (pre[j] = ix[home + j]): an answer within them costs no further round trip.
// The sweep steps load the whole 4-slot group of the home: a probe rarely
// runs past it, and a wave waits for its slowest lane.
template <int PH>
__device__ __forceinline__ int64_t find_slot_pre(const Idx* __restrict__ ix, uint64_t H, uint64_t key, uint64_t home,
                                                 const Idx (&pre)[PH], uint64_t* first_free, Idx* out) {
  const uint64_t mask = H - 1;
#pragma unroll
  for (int j = 0; j < PH; ++j) {
    const uint64_t t = (home + j) & mask;
    if (pre[j].key == key) {
      *out = pre[j];
      return static_cast<int64_t>(t);
    }
    if (pre[j].key == EMPTY_KEY) {
      *first_free = t;
      return -1;
    }
  }
  return probe_past(ix, H, key, (home + PH - 1) & mask, PH, first_free, out);
}

// Index `key` (known to be absent) under entry id `id`, starting the linear
// probe at `start`: the key is claimed with a compare-and-swap on an EMPTY
// slot, then the id is written.  Returns false when the index is full.
__device__ __forceinline__ bool index_insert(Idx* ix, uint64_t H, uint64_t key, uint64_t start, uint32_t id) {
  if (start >= H) return false;
  const uint64_t mask = H - 1;
  uint64_t s = start;
  for (uint64_t i = 0; i < H; ++i, s = (s + 1) & mask) {
    if (ix[s].key != EMPTY_KEY) continue;
    const unsigned long long old = atomicCAS(reinterpret_cast<unsigned long long*>(&ix[s].key),
                                             static_cast<unsigned long long>(EMPTY_KEY),
                                             static_cast<unsigned long long>(key));
    if (old == EMPTY_KEY) {
      ix[s].id = id;
      return true;
    }
  }
  return false;
}

// Presence filter of the index (a blocked Bloom filter): one 64-bit word per
// 8 index slots, three bits of one word per key.  While the filter is valid
// every key the index holds (alive or dead entry alike) has its bits set, so
// a key with any of its bits clear is not in the index and its probe needs no
// index read.  The word comes from bits 32 and up of the key's hash (the
// index home from the low bits), the bits from a second multiplicative hash
// of it.  It is cleared with the index and filled by every kernel that
// inserts keys while it is kept (the host tracks whether it is: steps without
// it leave it stale until it is rebuilt from the entries).
struct PfPos {
  uint64_t w, bits;
};
__device__ __forceinline__ PfPos pf_pos(uint64_t key, uint64_t nw) {
  const uint64_t m = mix64(key);
  const uint64_t q = m * 0x9e3779b97f4a7c15ull;
  return PfPos{(m >> 32) & (nw - 1), (1ull << (q >> 58)) | (1ull << ((q >> 52) & 63)) | (1ull << ((q >> 46) & 63))};
}
// the key's bits into member b's filter, if there is one (after the key entered the index)
__device__ __forceinline__ void pf_add(const Pf& pf, int b, uint64_t key) {
  if (!pf.w) return;
  const PfPos p = pf_pos(key, pf.n);
  atomicOr(reinterpret_cast<unsigned long long*>(pf.w + b * pf.stride + p.w), static_cast<unsigned long long>(p.bits));
}

// Entries of every arena of member b when the forward launch that runs step
// k began (lane a holds arena a): the counts of the launch before it plus its
// appends.  That launch began at step k-1, or at k-2 when it applied steps
// k-2 and k-1 together (no launch began at k-1 then).  For k = 1 the counts
// of the sweep's start.  Appends past an arena's capacity A were refused (the
// table-full flag fails the call), so counts are cut at A: no scan leaves its
// arena.
__device__ __forceinline__ uint32_t counts_before(const StepArr& sa, int b, int k, uint64_t A) {
  const int lane = threadIdx.x & 63;
  const int64_t row = static_cast<int64_t>(b) * sa.nstride;
  const uint32_t n1 = sa.nb[(row + k - 1) * NA + lane], a1 = sa.app[(row + k - 1) * NA + lane];
  uint64_t n;
  if (k < 2) {
    n = static_cast<uint64_t>(n1) + a1;
  } else {
    const uint32_t n2 = sa.nb[(row + k - 2) * NA + lane], a2 = sa.app[(row + k - 2) * NA + lane];
    n = n1 != NB_UNSET ? static_cast<uint64_t>(n1) + a1 : static_cast<uint64_t>(n2) + a2;
  }
  return static_cast<uint32_t>(n < A ? n : A);
}

// Entries of every arena of member b after forward step k (lane a: arena a).
__device__ __forceinline__ uint32_t counts_after(const StepArr& sa, int b, int k, uint64_t A) {
  return counts_before(sa, b, k + 1, A);
}

// Entries the reverse sweep must scan to undo step k: those created by the
// forward launches up to the one that applied step k, i.e. the counts when the
// next forward launch began (at k + 1, or k + 2 when k + 1 began no launch);
// nb[M + 1] holds the counts at the end of the forward sweep.
__device__ __forceinline__ uint32_t counts_reverse(const StepArr& sa, int b, int k, uint64_t A) {
  const int lane = threadIdx.x & 63;
  const int64_t row = static_cast<int64_t>(b) * sa.nstride;
  const uint32_t n1 = sa.nb[(row + k + 1) * NA + lane], n2 = sa.nb[(row + k + 2) * NA + lane];
  const uint64_t n = n1 != NB_UNSET ? n1 : n2;
  return static_cast<uint32_t>(n < A ? n : A);
}

// Arena of a block of an entry scan (blocks are NA-way interleaved over the
// arenas), the block's rank among those of its arena, and their number.
__device__ __forceinline__ int scan_arena() { return static_cast<int>(blockIdx.x & (NA - 1)); }
__device__ __forceinline__ uint64_t scan_rank() { return blockIdx.x / NA; }
__device__ __forceinline__ uint64_t scan_blocks() { return gridDim.x / NA; }

__device__ __forceinline__ uint32_t shard() { return blockIdx.x & (SH - 1); }
__device__ __forceinline__ uint32_t cshard() { return blockIdx.x & (CSH - 1); }

// index of the sharded per-step accumulators
__device__ __forceinline__ int64_t sidx(const StepArr& sa, int b, int sh, int64_t k) {
  return (static_cast<int64_t>(b) * SH + sh) * sa.stride + k;
}

__device__ __forceinline__ void count(Counters* cnt, int b, int which, unsigned long long v) {
  if (v) atomicAdd(&cnt[b].sh[cshard()].v[which], v);
}

template <class T>
__device__ __forceinline__ T fmaT(T a, T b, T c);
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) {
  return fmaf(a, b, c);
}
template <>
__device__ __forceinline__ double fmaT<double>(double a, double b, double c) {
  return fma(a, b, c);
}

// Entropy terms of one raw amplitude r: r^2 ln r^2 (0 for r = 0) and r^2.
__device__ __forceinline__ void ent_add(Fx& a, Fx& b, double r) {
  const double r2 = r * r;
  if (r2 > 0.0) a = fx_add(a, fx_from(r2 * log(r2)));
  b = fx_add(b, fx_from(r2));
}

// Wave totals of the entropy sums into step k's shard (sa.ea non-null).
__device__ __forceinline__ void ent_flush(const StepArr& sa, int b, int k, Fx a, Fx e) {
  a = wave_fx(a);
  e = wave_fx(e);
  if ((threadIdx.x & 63) == 0 && (fx_nonzero(a) || fx_nonzero(e))) {
    const int sh = (blockIdx.x * (BLK / 64) + (threadIdx.x >> 6)) & (ES - 1);
    const int64_t idx = (static_cast<int64_t>(b) * ES + sh) * sa.stride + k;
    fx3_atomic_add(&sa.ea[idx], a);
    fx3_atomic_add(&sa.eb[idx], e);
  }
}

// The SCAN_U slots s0, s0 + stride, ... of one pass of a sweep step (slots
// past the table read as empty).

// The SCAN_U entries j0, j0 + stride, ... of one pass of a sweep step in arena
// s, n of them valid (positions past n read as empty).
template <class T>
__device__ __forceinline__ void load_pass(const View<T>& v, uint64_t base, uint64_t n, uint64_t j0, uint64_t stride,
                                          Slot<T>* out) {
#pragma unroll
  for (int u = 0; u < SCAN_U; ++u) {
    const uint64_t j = j0 + u * stride;
    if (j < n) {
      out[u] = v.sl[base + j];
    } else {
      out[u].key = EMPTY_KEY;
      out[u].meta = DEAD;
    }
  }
}

// Renormalisation scale before step k (1-based): S_{k-1}, from S_{k-2} and the
// removed weight of step k-1.  Every wave computes it (its first SH lanes read
// the shards) with identical arithmetic: no LDS and no block barrier.
__device__ __forceinline__ double wave_scale(const StepArr& sa, int b, int k) {
  const int64_t base = static_cast<int64_t>(b) * sa.stride;
  double S = sa.scale[base + (k >= 2 ? k - 2 : 0)];
  if (k >= 2) {
    const int lane = threadIdx.x & 63;
    Fx w = fx_zero();
    unsigned long long c = 0;
    if (lane < SH) {
      w = fx3_value(sa.pw[sidx(sa, b, lane, k - 1)]);
      c = sa.pcnt[sidx(sa, b, lane, k - 1)];
    }
    w = wave_fx(w);
    c = wave_u64(c);
    if (c) {
      const double R = fx_to_d(w);
      const double nu2 = 1.0 - S * S * R;
      if (nu2 > 0.0) S = S / sqrt(nu2);
    }
  }
  return S;
}



// ---------------------------------------------------------------------------
// state set-up
// ---------------------------------------------------------------------------

// An empty state: every index slot free, every arena empty.
__global__ void k_fill(Tab t, Pf pf) {
  const int b = blockIdx.y;
  Idx* ix = t.idx + b * t.Hcap;
  for (uint64_t s = blockIdx.x * blockDim.x + threadIdx.x; s < t.H; s += gridDim.x * blockDim.x) {
    ix[s].key = EMPTY_KEY;
    ix[s].id = NO_ID;
    if (pf.w && s < pf.n) pf.w[b * pf.stride + s] = 0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x < NA) t.ac[b * NA + threadIdx.x] = 0u;
}

// Insert n determinants into an empty state: item i goes to arena i % NA at
// position i / NA (no counter to contend for), then into the index.  keys and
// amps of member b at b * stride; n < 0: member b's count is cnt[b].ncompact
// (the compact copies of its live entries).
template <class T>
__global__ void k_insert_list(Tab t, Counters* cnt, const uint64_t* __restrict__ keys,
                              const double* __restrict__ amps, int64_t n_fixed, uint64_t stride, Pf pf) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int64_t n = n_fixed >= 0 ? n_fixed : static_cast<int64_t>(cnt[b].ncompact);
  unsigned long long ok = 0;
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t key = keys[b * stride + i];
    const int a = static_cast<int>(i % NA);
    const uint64_t pos = static_cast<uint64_t>(i / NA);
    if (pos >= t.A) {
      atomicOr(&cnt[b].flags, F_TABLE_FULL);
      continue;
    }
    const uint64_t e = a * t.A + pos;
    v.sl[e].key = key;
    v.sl[e].amp = static_cast<T>(amps[b * stride + i]);
    v.sl[e].meta = 0u;
    v.born(e) = 0u;
    v.lam(e) = T(0);
    if (!index_insert(v.ix, v.H, key, home_slot(key, v.H), entry_id(a, pos))) {
      atomicOr(&cnt[b].flags, F_TABLE_FULL);
      continue;
    }
    pf_add(pf, b, key);
    ++ok;
  }
  if (blockIdx.x == 0 && threadIdx.x < NA) {
    const int64_t a = threadIdx.x;
    const int64_t m = n > a ? (n - a + NA - 1) / NA : 0;
    t.ac[b * NA + a] = static_cast<uint32_t>(m < static_cast<int64_t>(t.A) ? m : static_cast<int64_t>(t.A));
  }
  ok = wave_u64(ok);
  if ((threadIdx.x & 63) == 0 && ok) {
    count(cnt, b, C_LIVE, ok);
    count(cnt, b, C_OCC, ok);
  }
}

__global__ void k_trig(const double* __restrict__ theta, Trig* __restrict__ trig, int64_t M, int64_t ld,
                       Counters* cnt) {
  const int b = blockIdx.y;
  for (int64_t k = blockIdx.x * blockDim.x + threadIdx.x; k < M; k += gridDim.x * blockDim.x) {
    const double th = theta[b * M + k];
    if (!isfinite(th)) atomicOr(&cnt[0].flags, F_BAD_THETA);
    const double sh = sin(0.5 * th);
    Trig r;
    r.c = cos(th);
    r.s = sin(th);
    r.cm1 = -2.0 * sh * sh;
    trig[b * ld + k] = r;
  }
}

// Start of a sweep: every live entry becomes "born before the sweep"

// Start of a sweep: every live entry becomes "born before the sweep"
// (tag 0), dead entries get tag 0, per-step accumulators are cleared, and the
// arena counts of step 0 are the state's.
template <class T>
__global__ void k_sweep_begin(Tab t, StepArr sa, Counters* cnt, int64_t M) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  {
    const int a = scan_arena();
    const uint64_t n = t.ac[b * NA + a];
    for (uint64_t j = scan_rank() * BLK + threadIdx.x; j < n; j += scan_blocks() * BLK) {
      const uint64_t e = a * t.A + j;
      const uint32_t m = v.sl[e].meta;
      v.sl[e].meta = (m & DEAD) ? DEAD : 0u;
      v.born(e) = 0u;
    }
  }
  const uint64_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t gsz = gridDim.x * blockDim.x;
  const int64_t base = static_cast<int64_t>(b) * sa.stride;
  for (uint64_t i = gtid; i < static_cast<uint64_t>((M + 1) * SH); i += gsz) {
    const int sh = static_cast<int>(i / (M + 1));
    const int64_t k = static_cast<int64_t>(i % (M + 1));
    sa.pw[sidx(sa, b, sh, k)] = fx3_zero();
    sa.pcnt[sidx(sa, b, sh, k)] = 0u;
    if (sa.pvis) sa.pvis[sidx(sa, b, sh, k)] = 0u;
    sa.gacc[sidx(sa, b, sh, k)] = fx3_zero();
  }
  for (uint64_t i = gtid; i < static_cast<uint64_t>(M + 1); i += gsz) {
    sa.logn[base + i] = 0u;
    sa.scale[base + i] = cnt[b].S;  // steps that remove nothing keep the scale
  }
  for (uint64_t i = gtid; i < static_cast<uint64_t>((M + 3) * NA); i += gsz) {
    const int64_t row = static_cast<int64_t>(b) * sa.nstride * NA;
    sa.nb[row + i] = i < static_cast<uint64_t>(NA) ? t.ac[b * NA + i] : NB_UNSET;
    sa.app[row + i] = 0u;
  }
  if (sa.ea) {
    for (uint64_t i = gtid; i < static_cast<uint64_t>((M + 1) * ES); i += gsz) {
      const int64_t idx = (static_cast<int64_t>(b) * ES + static_cast<int64_t>(i / (M + 1))) * sa.stride +
                          static_cast<int64_t>(i % (M + 1));
      sa.ea[idx] = fx3_zero();
      sa.eb[idx] = fx3_zero();
    }
  }
  for (uint64_t i = gtid; i < static_cast<uint64_t>(sa.nws * WSTAT); i += gsz) sa.ws[b * sa.nws * WSTAT + i] = 0ull;
  for (uint64_t i = gtid; i < static_cast<uint64_t>(CSH); i += gsz) {
    cnt[b].sh[i].v[C_DU] = 0;
    cnt[b].sh[i].v[C_PAIRS] = 0;
    cnt[b].sh[i].v[C_INS] = 0;
    cnt[b].sh[i].v[C_PRUNED] = 0;
    cnt[b].sh[i].v[C_HITS] = 0;
  }
  if (gtid == 0) {
    cnt[b].logcnt = 0;
    if (b == 0) cnt[0].stop = ~0u;
  }
}

// End of a forward sweep, or of a run of its steps up to k_last (one block
// per state): the per-wave statistics folded into the state's counters, the
// arena counts after the last step that ran (a run stops early at the step a
// growth check stopped), and at the end of the sweep the final scale S_M and
// the counts the reverse sweep starts from (nb[M + 1]).
__global__ void k_sweep_end(Tab t, StepArr sa, Counters* cnt, int64_t M, int64_t k_last, const Sync* sy,
                            int fold_only) {
  const int b = blockIdx.x;
  if (threadIdx.x == 0 && sy && sy->timeout) atomicOr(&cnt[b].flags, F_TIMEOUT);
  if (M == 0) return;
  const double S = fold_only ? 0.0 : wave_scale(sa, b, static_cast<int>(M) + 1);
  unsigned long long tot[WSTAT];
  for (int i = 0; i < WSTAT; ++i) tot[i] = 0;
  for (int64_t w = threadIdx.x; w < sa.nws; w += blockDim.x)
#pragma unroll
    for (int i = 0; i < WSTAT; ++i) {
      tot[i] += sa.ws[(b * sa.nws + w) * WSTAT + i];
      sa.ws[(b * sa.nws + w) * WSTAT + i] = 0ull;  // folded: a later run starts from zero
    }
  // block totals: wave sums, then wave 0 adds the other waves' (LDS)
  __shared__ unsigned long long part[BLK / 64][WSTAT];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < WSTAT; ++i) tot[i] = wave_u64(tot[i]);
  if (lane == 0)
    for (int i = 0; i < WSTAT; ++i) part[wv][i] = tot[i];
  __syncthreads();
  for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w)
    for (int i = 0; i < WSTAT; ++i) tot[i] += part[w][i];
  if (wv != 0) return;
  // live count over the shards, before this fold
  unsigned long long live = lane < CSH ? cnt[b].sh[lane].v[C_LIVE] : 0ull;
  live = wave_u64(live);
  // arena counts after the last step that ran
  int64_t ke = M;
  if (fold_only) {
    const int64_t stop = static_cast<int64_t>(cnt[0].stop);
    ke = stop - 1 < k_last ? stop - 1 : k_last;
  }
  const uint32_t na = counts_after(sa, b, static_cast<int>(ke), t.A);
  t.ac[b * NA + lane] = na;
  if (!fold_only) {
    const int64_t row = (static_cast<int64_t>(b) * sa.nstride + M + 1) * NA;
    sa.nb[row + lane] = na;
    sa.app[row + lane] = 0u;
  }
  const unsigned long long nent = wave_u64(na);
  if (lane < CSH) cnt[b].sh[lane].v[C_OCC] = lane == 0 ? nent : 0ull;
  if (lane == 0) {
    if (!fold_only) {
      sa.scale[static_cast<int64_t>(b) * sa.stride + M] = S;
      cnt[b].S = S;
      if (sa.pvis) sa.pvis[sidx(sa, b, 0, 0)] = static_cast<uint32_t>(live + tot[3] - tot[4]);  // after the sweep
    }
    CShard& c0 = cnt[b].sh[0];
    c0.v[C_PRUNED] += tot[0];
    c0.v[C_DU] += tot[1];
    c0.v[C_PAIRS] += tot[2];
    c0.v[C_INS] += tot[3];
    c0.v[C_LIVE] += tot[3] - tot[4];
    c0.v[C_HITS] += tot[6];
  }
}


// ---------------------------------------------------------------------------
// forward step k: pair rotation exp(theta_k A_k) + truncation
// ---------------------------------------------------------------------------
// For a pair (L, U) with tau|L> = s|U> and amplitudes (x, y):
//   x' = x cos - s sin y,  y' = y cos + s sin x       (closed form, Eqs. 4-5)
// written as x' = x + (x (cos-1) - s sin y) for accuracy at small theta.
// Truncation (Methods section): a member whose |S x'| < thr is removed; its
// entry keeps x' for the reverse sweep.  The removed weight feeds the
// renormalisation scale of the next step.
//
// Arena for the entries a wave creates in step k: a hash of the wave and the
// step, so that the creations of any step spread over all arenas whatever
// arena the creating wave scans (a state that starts in one arena and doubles
// in a few steps would otherwise pile into a few arenas).
__device__ __forceinline__ int create_arena(int k) {
  const uint64_t w = static_cast<uint64_t>(blockIdx.x) * (BLK / 64) + (threadIdx.x >> 6);
  return static_cast<int>(mix64((static_cast<uint64_t>(k) << 32) | w) & (NA - 1));
}

// Positions for the new entries a wave creates in one round: lanes with
// want[u] get consecutive positions of the wave's arena after those taken
// before (one returning atomic per wave and round).  Every lane of the wave
// must be active.  Returns the arena; pos[u] is set for the lanes that want.
template <int U>
__device__ __forceinline__ int claim_positions(const StepArr& sa, int b, int k, uint32_t nk, const bool (&want)[U],
                                               uint64_t (&pos)[U]) {
  const int lane = threadIdx.x & 63;
  const int a = create_arena(k);
  unsigned long long m[U];
  uint32_t tot = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    m[u] = __ballot(want[u]);
    tot += static_cast<uint32_t>(__popcll(m[u]));
  }
  if (tot == 0) return a;
  uint32_t basep = 0;
  if (lane == 0) basep = atomicAdd(&sa.app[(static_cast<int64_t>(b) * sa.nstride + k) * NA + a], tot);
  basep = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(basep)));
  const uint32_t arena_start = static_cast<uint32_t>(__shfl(static_cast<int>(nk), a, 64));
  const unsigned long long below = lane ? ((1ull << lane) - 1ull) : 0ull;
  uint32_t run = arena_start + basep;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    pos[u] = run + static_cast<uint32_t>(__popcll(m[u] & below));
    run += static_cast<uint32_t>(__popcll(m[u]));
  }
  return a;
}

// PF: partners are looked up in the presence filter first, and in the index
// only when the filter may hold them.
template <class T, bool ENT, bool PF = false>
__device__ __forceinline__ void fwd_step(const Tab& t, const FacMask* __restrict__ fac,
                                         const Trig* __restrict__ trig, int64_t ld, const StepArr& sa, Counters* cnt,
                                         const LogArr& lg, int k, double thr, int prune_all, int log_on,
                                         uint64_t occ_lim, int b0, int nmem, const Pf& pf = Pf{}) {
  const int b = blockIdx.y + b0;  // b0: the member of a launch for one member (nmem members in all)
  const View<T> v = view<T>(t, b);
  const uint64_t* pfm = PF ? pf.w + b * pf.stride : nullptr;  // the member's filter words
  // the factor first: its loads then overlap everything the step loads next
  const FacMask f = fac[k - 1];
  const Trig tr = trig[b * ld + k - 1];
  const T sn = static_cast<T>(tr.s), cm1 = static_cast<T>(tr.cm1);
  const uint64_t pm = f.occ | f.vir;
  const int64_t base = static_cast<int64_t>(b) * sa.stride;
  const int lane = threadIdx.x & 63;
  const uint32_t K = static_cast<uint32_t>(k);
  const int s = scan_arena();
  // entries of every arena when the launch began (lane a: arena a)
  const uint32_t nk = counts_before(sa, b, k, v.A);
  if (occ_lim != NO_LIMIT) {
    // Growth check: every block of every member sees the same exact counts,
    // so all return together when a member's index holds more than the limit
    // (the host grows the index and runs the step again); a step that runs
    // at most doubles the entries, so the index stays below twice the limit.
    // The steps after one that returned return too: they see its counts
    // (counts_before falls back to the step before) or, further on, counts
    // clamped to the arena size, far above any limit.
    unsigned long long most = 0;
    for (int bb = 0; bb < nmem; ++bb) {
      const unsigned long long n = wave_u64(bb == b ? nk : counts_before(sa, bb, k, v.A));
      most = n > most ? n : most;
    }
    if (most > occ_lim) {
      if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(&cnt[0].stop, K);
      return;
    }
  }
  const uint64_t ns = static_cast<uint32_t>(__shfl(static_cast<int>(nk), s, 64));  // this block's arena
  if (scan_rank() == 0 && threadIdx.x == 0) sa.nb[(static_cast<int64_t>(b) * sa.nstride + k) * NA + s] = static_cast<uint32_t>(ns);
  // this wave's statistics slot (read now, written back at the end)
  unsigned long long* wst = sa.ws + (static_cast<int64_t>(b) * sa.nws + (blockIdx.x * (BLK / 64) + (threadIdx.x >> 6))) * WSTAT;
  const unsigned long long wold = lane < WSTAT ? wst[lane] : 0ull;

  // SCAN_U entries per lane per pass.  The first pass's entries are requested
  // before the scale is reduced, and each pass requests the next pass's before
  // it probes partners, so a lane keeps two passes of loads in flight.  (An
  // entry read early is safe for the same reason a partner's is: whatever
  // other lanes write during the step keeps its presence at the start of the
  // step, and the owner of its pair, unchanged.)  The pass loop runs the same
  // number of times for every lane of a wave.
  const uint64_t ebase = s * v.A;
  const uint64_t stride = scan_blocks() * BLK;
  const uint64_t pass = SCAN_U * stride;
  const uint64_t j0w = scan_rank() * BLK + (threadIdx.x & ~63u);  // the wave's first position
  uint64_t j0 = scan_rank() * BLK + threadIdx.x;
  Slot<T> nxt[SCAN_U];
  load_pass<T>(v, ebase, ns, j0, stride, nxt);

  // threshold 0 never truncates, so the scale is not needed
  const bool trunc = thr > 0.0;
  const double S = trunc ? wave_scale(sa, b, k) : 1.0;
  if (trunc && k >= 2 && blockIdx.x == 0 && threadIdx.x == 0) sa.scale[base + k - 1] = S;


  Red r;
  r.f = fx_zero();
  for (int i = 0; i < 7; ++i) r.c[i] = 0;
  // c[0] removed count, c[1] visits, c[2] pairs, c[3] creates, c[4] kills, c[5] new entries,
  // c[6] pairs whose partner existed
  unsigned int flags = 0;

  auto kill = [&](uint64_t e, T x) {
    v.sl[e].amp = x;
    v.sl[e].meta = DEAD | K;
    const double dv = static_cast<double>(x);
    r.f = fx_add(r.f, fx_from(dv * dv));
    r.c[0] += 1;
    r.c[4] += 1;
  };
  auto drop_new = [&](T x) {  // created and truncated in the same step
    const double dv = static_cast<double>(x);
    r.f = fx_add(r.f, fx_from(dv * dv));
    r.c[0] += 1;
  };
  // revive the dead entry e (`old` its contents) of determinant `key` with value x
  auto revive = [&](uint64_t key, T x, uint64_t e, const Slot<T>& old) {
    if ((old.meta & TAG) != 0u && log_on) {  // dead entry of this sweep: remember it
      const unsigned long long p = atomicAdd(&cnt[b].logcnt, 1ull);
      if (p < lg.cap) {
        const uint64_t li = b * lg.cap + p;
        lg.key[li] = key;
        lg.meta[li] = old.meta;
        lg.born[li] = v.born(e);
        static_cast<T*>(lg.amp)[li] = old.amp;
        atomicAdd(&sa.logn[base + k], 1u);
      } else {
        flags |= F_LOG_FULL;
      }
    }
    v.sl[e].amp = x;
    v.born(e) = K;
    v.sl[e].meta = K;
    r.c[3] += 1;
  };

  Fx ent_a = fx_zero(), ent_b = fx_zero();  // entropy sums (when tracked)
  for (uint64_t jw = j0w; jw < ns; jw += pass, j0 += pass) {
    Slot<T> mes[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) mes[u] = nxt[u];
    if (jw + pass < ns) load_pass<T>(v, ebase, ns, j0 + pass, stride, nxt);
    // the home index slots of this pass's partners are then loaded together
    // (with the filter: their filter words, then the index groups of the
    // partners the filter may hold)
    uint64_t home[SCAN_U];
    Idx hv[SCAN_U][4];
    bool act[SCAN_U], look[SCAN_U];
    uint64_t pfw[SCAN_U], pfb[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      const Slot<T>& me = mes[u];
      act[u] = false;
      if (me.key == EMPTY_KEY) continue;
      const uint32_t m = me.meta;
      if (m & DEAD) {
        // removed by its pair's owner earlier in this step: it was live when
        // the step began, so it counts as visited
        if ((m & TAG) == K) r.c[1] += 1;
        continue;
      }
      if ((m & TAG) == K) continue;  // revived in this step
      r.c[1] += 1;
      const bool lower = ((me.key & f.occ) == f.occ) && !(me.key & f.vir);
      const bool upper = ((me.key & f.vir) == f.vir) && !(me.key & f.occ);
      if (!lower && !upper) {
        if (prune_all && !(fabs(S * static_cast<double>(me.amp)) >= thr)) {
          kill(ebase + j0 + u * stride, me.amp);
        } else if (ENT) {
          ent_add(ent_a, ent_b, static_cast<double>(me.amp));
        }
        continue;
      }
      act[u] = true;
      home[u] = home_slot(me.key ^ pm, v.H);
      if (PF) {
        const PfPos p = pf_pos(me.key ^ pm, pf.n);
        pfw[u] = pfm[p.w];
        pfb[u] = p.bits;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) hv[u][i] = v.ix[(home[u] + i) & (v.H - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      look[u] = act[u];
      if (PF) {
        look[u] = act[u] && (pfw[u] & pfb[u]) == pfb[u];
        if (act[u] && !look[u]) {
          // the partner is absent, so the pair creates it when its new value
          // (the rotation of this member's amplitude alone) is kept: that
          // needs a free index slot, so its index group is loaded as well
          const T ss = (__popcll(mes[u].key & f.sgn) & 1) ? -sn : sn;
          look[u] = fabs(S * static_cast<double>(static_cast<T>(ss * mes[u].amp))) >= thr;
        }
        if (look[u]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) hv[u][i] = v.ix[(home[u] + i) & (v.H - 1)];
        }
      }
    }
    // resolve the probes, then load the partners' entries together
    uint64_t free_start[SCAN_U], pe[SCAN_U];
    bool found[SCAN_U];
    Slot<T> pv[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      found[u] = false;
      free_start[u] = v.H;
      if (!look[u]) continue;
      Idx iv;
      found[u] = find_slot_pre<4>(v.ix, v.H, mes[u].key ^ pm, home[u], hv[u], &free_start[u], &iv) >= 0;
      if (found[u]) {
        if (iv.id == NO_ID) {  // cannot happen: only this lane creates its partner
          flags |= F_INCONSISTENT;
          found[u] = false;
        } else {
          pe[u] = v.off(iv.id);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u)
      if (found[u]) pv[u] = v.sl[pe[u]];
    // One pair: the new values, the keep decisions, the member updates.  A
    // lane whose partner is absent needs no partner data, so those lanes go
    // first, while the partners' entries load: the new entries they create
    // claim their index slots and arena positions with returning atomics
    // that are then in flight together with those loads.
    bool want[SCAN_U];
    uint64_t wkey[SCAN_U], wfree[SCAN_U];
    T wamp[SCAN_U];
    auto pair_step = [&](int u) {
      const Slot<T>& me = mes[u];
      const uint64_t e = ebase + j0 + u * stride;
      const uint64_t key = me.key;
      const bool lower = ((key & f.occ) == f.occ) && !(key & f.vir);
      const uint64_t pk = key ^ pm;
      bool p_alive = false, p_start = false;
      if (found[u]) {
        p_alive = !(pv[u].meta & DEAD);
        p_start = p_alive || ((pv[u].meta & TAG) == K);
      }
      if (!lower && p_start) return;  // the lower member owns the pair
      r.c[2] += 1;
      if (lower && p_alive) r.c[6] += 1;
      const T ss = (__popcll(key & f.sgn) & 1) ? -sn : sn;
      const T x = lower ? me.amp : T(0);
      const T y = lower ? (p_alive ? pv[u].amp : T(0)) : me.amp;
      const T xn = x + fmaT<T>(x, cm1, -ss * y);
      const T yn = y + fmaT<T>(y, cm1, ss * x);
      const bool keepx = fabs(S * static_cast<double>(xn)) >= thr;
      const bool keepy = fabs(S * static_cast<double>(yn)) >= thr;
      if (ENT) {  // the pair's members that stay live after the step
        if (keepx) ent_add(ent_a, ent_b, static_cast<double>(xn));
        if (keepy) ent_add(ent_a, ent_b, static_cast<double>(yn));
      }
      // the partner's new value, when it is created (kept, and not present)
      bool make = false;
      T pnew = T(0);
      if (lower) {
        if (keepx) v.sl[e].amp = xn; else kill(e, xn);
        if (p_alive) {
          if (keepy) v.sl[pe[u]].amp = yn; else kill(pe[u], yn);
        } else if (keepy) {
          make = true;
          pnew = yn;
        } else {
          drop_new(yn);
        }
      } else {
        if (keepy) v.sl[e].amp = yn; else kill(e, yn);
        if (keepx) {
          make = true;
          pnew = xn;
        } else {
          drop_new(xn);
        }
      }
      if (make) {
        if (found[u]) {
          revive(pk, pnew, pe[u], pv[u]);  // its dead entry comes back
        } else {
          want[u] = true;                   // a new entry (positions below)
          wkey[u] = pk;
          wamp[u] = pnew;
          wfree[u] = free_start[u];
        }
      }
    };
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      want[u] = false;
      if (act[u] && !found[u]) pair_step(u);
    }
    // new entries: each claims the free index slot its probe ended at (a
    // compare-and-swap of the key) while the wave claims positions in its
    // arena, so the two returning atomics overlap; then the entries, and the
    // entry ids into the index slots.  Until its id is written a claimed slot
    // is seen by no probe of this step but its own: a created key is the
    // partner of one scanned entry only.  (With the filter every creating
    // lane has probed its index group; the insert from the home covers a lane
    // that did not.)
    bool slot_ok[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      slot_ok[u] = false;
      if (want[u] && wfree[u] < v.H)
        slot_ok[u] = atomicCAS(reinterpret_cast<unsigned long long*>(&v.ix[wfree[u]].key),
                               static_cast<unsigned long long>(EMPTY_KEY),
                               static_cast<unsigned long long>(wkey[u])) == EMPTY_KEY;
    }
    uint64_t pos[SCAN_U];
    const int a = claim_positions<SCAN_U>(sa, b, k, nk, want, pos);
    // the pairs whose partner is present, once its entry has arrived
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u)
      if (act[u] && found[u]) pair_step(u);
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      if (!want[u]) continue;
      if (pos[u] >= v.A) {  // the sweep fails ("hash table full")
        flags |= F_TABLE_FULL;
        continue;
      }
      const uint64_t e = a * v.A + pos[u];
      v.sl[e].key = wkey[u];
      v.sl[e].amp = wamp[u];
      v.sl[e].meta = K;
      v.born(e) = K;
      v.lam(e) = T(0);
      // (a slot another new key took first: the probe goes on past it)
      if (slot_ok[u]) {
        v.ix[wfree[u]].id = entry_id(a, pos[u]);
      } else if (!index_insert(v.ix, v.H, wkey[u],
                               PF && !look[u] ? home[u] : wfree[u] < v.H ? (wfree[u] + 1) & (v.H - 1) : v.H,
                               entry_id(a, pos[u]))) {
        flags |= F_TABLE_FULL;
        continue;
      }
      if (PF) pf_add(pf, b, wkey[u]);
      r.c[3] += 1;
      r.c[5] += 1;
    }
  }

  if (flags) atomicOr(&cnt[b].flags, flags);
  if (ENT) ent_flush(sa, b, k, ent_a, ent_b);
  // wave totals: statistics go to the wave's private slot (plain stores, no
  // block barrier); removed weight, when there is any, to a sharded atomic
  unsigned int c[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) c[i] = wave_u32(static_cast<unsigned int>(r.c[i]));
  const int wsh = (blockIdx.x * (BLK / 64) + (threadIdx.x >> 6)) & (SH - 1);
  if (c[0]) {
    const Fx w = wave_fx(r.f);
    if (lane == 0) {
      fx3_atomic_add(&sa.pw[sidx(sa, b, wsh, k)], w);
      atomicAdd(&sa.pcnt[sidx(sa, b, wsh, k)], c[0]);
    }
  }
  if (sa.pvis && c[1] && lane == 0) atomicAdd(&sa.pvis[sidx(sa, b, wsh, k)], c[1]);
  if (lane < 7) {
    const unsigned int mine = lane == 0 ? c[0] : lane == 1 ? c[1] : lane == 2 ? c[2] : lane == 3 ? c[3]
                              : lane == 4 ? c[4] : lane == 5 ? c[5] : c[6];
    wst[lane] = wold + mine;
  }
}


// ---------------------------------------------------------------------------
// reverse step k: exact inverse of the truncated forward step on psi, and
// the adjoint update  w = U_k^T lambda_k,  g_k = <w|A_k psi_{k-1}>,
// lambda_{k-1} = P_{k-1} w  (raw, unnormalised amplitudes; the
// renormalisation constants cancel in the Rayleigh quotient).
// ---------------------------------------------------------------------------
// "Present after step k": alive, or dead with tag k (removed by the
// truncation of step k; its entry holds the pre-truncation value and its
// adjoint component is 0).  Pair inversion:
//   both present            (x, y) = U^T (x', y')
//   only one present        the other was created and truncated in step k:
//                           x = x' / cos (or y = y' / cos)
// Members born in step k are removed; entries that died in step k are
// revived.  Only the entries that existed after step k are scanned (those
// created by later steps lie beyond the counts of the next forward launch).
template <class T, bool PF = false>
__device__ __forceinline__ void rev_step(const Tab& t, const FacMask* __restrict__ fac,
                                         const Trig* __restrict__ trig, int64_t ld, const StepArr& sa, Counters* cnt,
                                         int k, int b0, const Pf& pf = Pf{}) {
  const int b = blockIdx.y + b0;  // b0: the member of a launch for one member
  const View<T> v = view<T>(t, b);
  const uint64_t* pfm = PF ? pf.w + b * pf.stride : nullptr;  // the member's filter words
  const int s = scan_arena();
  const uint64_t ns = static_cast<uint32_t>(__shfl(static_cast<int>(counts_reverse(sa, b, k, v.A)), s, 64));

  const FacMask f = fac[k - 1];
  const Trig tr = trig[b * ld + k - 1];
  const T c = static_cast<T>(tr.c), sn = static_cast<T>(tr.s), cm1 = static_cast<T>(tr.cm1);
  const uint64_t pm = f.occ | f.vir;
  const uint32_t K = static_cast<uint32_t>(k);

  Red r;
  r.f = fx_zero();
  for (int i = 0; i < 7; ++i) r.c[i] = 0;
  unsigned int flags = 0;

  // SCAN_U entries per lane per pass, the next pass's requested before this
  // pass probes partners (as in the forward step)
  const uint64_t ebase = s * v.A;
  const uint64_t stride = scan_blocks() * BLK;
  const uint64_t pass = SCAN_U * stride;
  Slot<T> nxt[SCAN_U];
  load_pass<T>(v, ebase, ns, scan_rank() * BLK + threadIdx.x, stride, nxt);
  for (uint64_t j0 = scan_rank() * BLK + threadIdx.x; j0 < ns; j0 += pass) {
    Slot<T> mes[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) mes[u] = nxt[u];
    if (j0 + pass < ns) load_pass<T>(v, ebase, ns, j0 + pass, stride, nxt);
    uint64_t home[SCAN_U];
    Idx hv[SCAN_U][4];
    T lms[SCAN_U];
    bool act[SCAN_U], look[SCAN_U];
    uint64_t pfw[SCAN_U], pfb[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      const Slot<T>& me = mes[u];
      act[u] = false;
      if (me.key == EMPTY_KEY) continue;
      const uint32_t m = me.meta;
      const bool dead = (m & DEAD) != 0u;
      if (dead && (m & TAG) != K) continue;
      const bool lower = ((me.key & f.occ) == f.occ) && !(me.key & f.vir);
      const bool upper = ((me.key & f.vir) == f.vir) && !(me.key & f.occ);
      const uint64_t e = ebase + j0 + u * stride;
      if (!lower && !upper) {
        if (dead) {  // truncated at step k without being rotated (first step of a sweep)
          v.sl[e].meta = v.born(e);
          v.lam(e) = T(0);
        }
        continue;
      }
      act[u] = true;
      // the adjoint value of this member (only members of a pair need it)
      // and the partner's home index slot; the partner's adjoint value is
      // loaded only by the pair's owner once the partner is found
      lms[u] = v.lam_pre(e);
      home[u] = home_slot(me.key ^ pm, v.H);
      if (PF) {
        const PfPos p = pf_pos(me.key ^ pm, pf.n);
        pfw[u] = pfm[p.w];
        pfb[u] = p.bits;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) hv[u][i] = v.ix[(home[u] + i) & (v.H - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      look[u] = act[u];
      if (PF) {
        look[u] = act[u] && (pfw[u] & pfb[u]) == pfb[u];
        if (look[u]) {
#pragma unroll
          for (int i = 0; i < 4; ++i) hv[u][i] = v.ix[(home[u] + i) & (v.H - 1)];
        }
      }
    }
    // resolve the probes, then load the partners' entries together
    bool found[SCAN_U];
    uint64_t pe[SCAN_U];
    Slot<T> pv[SCAN_U];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      found[u] = false;
      if (!look[u]) continue;
      uint64_t ff = v.H;
      Idx iv;
      found[u] = find_slot_pre<4>(v.ix, v.H, mes[u].key ^ pm, home[u], hv[u], &ff, &iv) >= 0;
      if (found[u]) {
        if (iv.id == NO_ID) {
          flags |= F_INCONSISTENT;
          found[u] = false;
        } else {
          pe[u] = v.off(iv.id);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u)
      if (found[u]) pv[u] = v.sl[pe[u]];
#pragma unroll
    for (int u = 0; u < SCAN_U; ++u) {
      if (!act[u]) continue;
      const Slot<T>& me = mes[u];
      const uint64_t e = ebase + j0 + u * stride;
      const uint32_t m = me.meta;
      const bool dead = (m & DEAD) != 0u;
      const uint64_t key = me.key;
      const bool lower = ((key & f.occ) == f.occ) && !(key & f.vir);
      bool p_pres = false;
      if (found[u]) p_pres = !(pv[u].meta & DEAD) || ((pv[u].meta & TAG) == K);
      if (!lower && p_pres) continue;  // the lower member owns the pair
      const T ss = (__popcll(key & f.sgn) & 1) ? -sn : sn;

      uint64_t eL = 0, eU = 0;
      uint32_t mL = 0, mU = 0;
      bool hL, hU;
      T xp, yp, lL, lU;
      if (lower) {
        eL = e; mL = m; hL = true;
        eU = pe[u]; mU = pv[u].meta; hU = p_pres;
        xp = me.amp;
        yp = hU ? pv[u].amp : T(0);
        lL = dead ? T(0) : v.lam_fin(me, lms[u]);
        lU = (hU && !(mU & DEAD)) ? v.lam_of(pv[u], eU) : T(0);
      } else {
        eU = e; mU = m; hU = true;
        hL = false;
        xp = T(0);
        yp = me.amp;
        lL = T(0);
        lU = dead ? T(0) : v.lam_fin(me, lms[u]);
      }
      const T wL = lL + fmaT<T>(lL, cm1, ss * lU);
      const T wU = lU + fmaT<T>(lU, cm1, -ss * lL);
      T x, y;
      if (hL && hU) {
        x = xp + fmaT<T>(xp, cm1, ss * yp);
        y = yp + fmaT<T>(yp, cm1, -ss * xp);
      } else if (hL) {
        x = xp / c;
        y = T(0);
      } else {
        x = T(0);
        y = yp / c;
      }
      const double sgn = (__popcll(key & f.sgn) & 1) ? -1.0 : 1.0;
      const double term = sgn * (static_cast<double>(wU) * static_cast<double>(x) -
                                 static_cast<double>(wL) * static_cast<double>(y));
      r.f = fx_add(r.f, fx_from(term));
      r.c[2] += 1;
      if (hL) {
        const uint32_t bL = (mL & DEAD) ? v.born(eL) : (mL & TAG);
        if (bL == K) {
          if (!hU) flags |= F_INCONSISTENT;
          v.sl[eL].meta = DEAD | K;
          r.c[4] += 1;
        } else {
          v.sl[eL].amp = x;
          v.lam(eL) = wL;
          v.sl[eL].meta = bL;
        }
      }
      if (hU) {
        const uint32_t bU = (mU & DEAD) ? v.born(eU) : (mU & TAG);
        if (bU == K) {
          if (!hL) flags |= F_INCONSISTENT;
          v.sl[eU].meta = DEAD | K;
          r.c[4] += 1;
        } else {
          v.sl[eU].amp = y;
          v.lam(eU) = wU;
          v.sl[eU].meta = bU;
        }
      }
    }
  }
  if (flags) atomicOr(&cnt[b].flags, flags);
  // wave total of the gradient dot product -> sharded exact accumulator
  const Fx g = wave_fx(r.f);
  const int wsh = (blockIdx.x * (BLK / 64) + (threadIdx.x >> 6)) & (SH - 1);
  if ((threadIdx.x & 63) == 0 && fx_nonzero(g)) fx3_atomic_add(&sa.gacc[sidx(sa, b, wsh, k)], g);
}

// Entries whose dead state a revival in forward step k overwrote get that
// state back once the reverse sweep has undone step k.
template <class T>
__device__ __forceinline__ void restore_step(const Tab& t, const LogArr& lg, const StepArr& sa, int k) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int64_t base = static_cast<int64_t>(b) * sa.stride;
  const uint32_t n = sa.logn[base + k];
  const uint32_t off = sa.logoff[base + k];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t li = b * lg.cap + off + i;
    // the determinant is still in the state (removed by the reverse step, so
    // dead); locate its entry by key
    uint64_t ff;
    Idx iv;
    if (find_slot(v.ix, v.H, lg.key[li], &ff, &iv) < 0 || iv.id == NO_ID) continue;
    const uint64_t e = v.off(iv.id);
    v.sl[e].meta = lg.meta[li];
    v.born(e) = lg.born[li];
    v.sl[e].amp = static_cast<const T*>(lg.amp)[li];
  }
}

// one launch per step.  ENT: the entropy sums are tracked (a separate
// instantiation keeps their registers out of the common case).
template <class T, bool ENT>
__global__ __launch_bounds__(BLK) void k_fwd(Tab t, const FacMask* __restrict__ fac,
                                                   const Trig* __restrict__ trig, int64_t ld, StepArr sa,
                                                   Counters* cnt, LogArr lg, int k, double thr, int prune_all,
                                                   int log_on, uint64_t occ_lim, int b0, int nmem) {
  fwd_step<T, ENT>(t, fac, trig, ld, sa, cnt, lg, k, thr, prune_all, log_on, occ_lim, b0, nmem);
}

template <class T>
__global__ __launch_bounds__(BLK) void k_rev(Tab t, const FacMask* __restrict__ fac, const Trig* __restrict__ trig,
                                             int64_t ld, StepArr sa, Counters* cnt, int k, int b0) {
  rev_step<T>(t, fac, trig, ld, sa, cnt, k, b0);
}

// The step kernels with the presence-filter probes (large states whose
// partners are nearly always absent; see pf_pos).
template <class T>
__global__ __launch_bounds__(BLK) void k_fwd_pf(Tab t, const FacMask* __restrict__ fac, const Trig* __restrict__ trig,
                                                int64_t ld, StepArr sa, Counters* cnt, LogArr lg, int k, double thr,
                                                int prune_all, int log_on, uint64_t occ_lim, int b0, int nmem, Pf pf) {
  fwd_step<T, false, true>(t, fac, trig, ld, sa, cnt, lg, k, thr, prune_all, log_on, occ_lim, b0, nmem, pf);
}

template <class T>
__global__ __launch_bounds__(BLK) void k_rev_pf(Tab t, const FacMask* __restrict__ fac, const Trig* __restrict__ trig,
                                                int64_t ld, StepArr sa, Counters* cnt, int k, int b0, Pf pf) {
  rev_step<T, true>(t, fac, trig, ld, sa, cnt, k, b0, pf);
}

// The forward step built for three resident waves per SIMD instead of two
// (fewer registers, a few spilled), so that more loads are in flight on each
// compute unit.  It pays once the state spans many passes of the grid; small
// states keep the build above, whose launches are chains of dependent loads
// that the spills would lengthen.  (A reverse build for four waves per SIMD
// gained at 32 qubits and lost at 48: the reverse keeps one build.)
template <class T>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(3))) void k_fwd_ho(
    Tab t, const FacMask* __restrict__ fac, const Trig* __restrict__ trig, int64_t ld, StepArr sa, Counters* cnt,
    LogArr lg, int k, double thr, int prune_all, int log_on, uint64_t occ_lim, int b0, int nmem) {
  fwd_step<T, false>(t, fac, trig, ld, sa, cnt, lg, k, thr, prune_all, log_on, occ_lim, b0, nmem);
}

template <class T>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(3))) void k_fwd_ho_pf(
    Tab t, const FacMask* __restrict__ fac, const Trig* __restrict__ trig, int64_t ld, StepArr sa, Counters* cnt,
    LogArr lg, int k, double thr, int prune_all, int log_on, uint64_t occ_lim, int b0, int nmem, Pf pf) {
  fwd_step<T, false, true>(t, fac, trig, ld, sa, cnt, lg, k, thr, prune_all, log_on, occ_lim, b0, nmem, pf);
}


// ---------------------------------------------------------------------------
// two factors per launch (threshold 0)
// ---------------------------------------------------------------------------
// With no truncation there is no global reduction between steps k and k+1, so
// one launch can apply both.  The determinants D, D^m1, D^m2, D^m1^m2 (m the
// XOR masks of the two factors, m1 != m2) are closed under both pair maps.
// Which pairs act follows from the keys alone: factor 1 pairs (0,1) and
// (2,3), factor 2 pairs (0,2) and (1,3), each when its members are lower/
// upper for that factor.  A lane whose determinant lies in a connected set
// of acting pairs looks up the other members of the set; the member with the
// smallest key among those present when the launch starts applies step k,
// then step k+1, to the whole set, with the same per-pair arithmetic, in the
// same order, as two single-step launches (results are bit-identical).  A
// member whose entry this launch created is recognised from its id (a
// position at or past its arena's count when the launch began), so no lane
// reads an entry another lane may still be writing.

__device__ __forceinline__ int side(uint64_t x, const FacMask& f) {
  if ((x & f.occ) == f.occ && !(x & f.vir)) return 1;   // lower
  if ((x & f.vir) == f.vir && !(x & f.occ)) return -1;  // upper
  return 0;
}

struct Quad {
  uint64_t q[4];
  bool e1a, e1b, e2a, e2b;  // acting pairs: f1 (0,1), (2,3); f2 (0,2), (1,3)
  unsigned comp;            // members connected to member 0 (bit mask)
};

__device__ __forceinline__ Quad make_quad(uint64_t X, uint64_t m1, uint64_t m2, const FacMask& f1,
                                          const FacMask& f2) {
  Quad Q;
  Q.q[0] = X;
  Q.q[1] = X ^ m1;
  Q.q[2] = X ^ m2;
  Q.q[3] = X ^ m1 ^ m2;
  Q.e1a = side(Q.q[0], f1) != 0;
  Q.e1b = side(Q.q[2], f1) != 0;
  Q.e2a = side(Q.q[0], f2) != 0;
  Q.e2b = side(Q.q[1], f2) != 0;
  unsigned c = 1u;
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    if (Q.e1a && (c & 3u)) c |= 3u;
    if (Q.e1b && (c & 12u)) c |= 12u;
    if (Q.e2a && (c & 5u)) c |= 5u;
    if (Q.e2b && (c & 10u)) c |= 10u;
  }
  Q.comp = c;
  return Q;
}

// An entry id created by the current launch: its position is at or past its
// arena's count when the launch began (arena_n: the block's LDS copy of the
// counts; a lane shuffle would read other lanes' registers, which is not
// defined for lanes that branched away).
__device__ __forceinline__ bool created_here(uint32_t id, const uint32_t* arena_n) {
  return (id & ID_POS_MASK) >= arena_n[id >> ID_POS_BITS];
}

template <class T, int PH>
__global__ __launch_bounds__(BLK) void k_fwd2(Tab t, const FacMask* __restrict__ fac, const Trig* __restrict__ trig,
                                              int64_t ld, StepArr sa, Counters* cnt, int k) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int lane = threadIdx.x & 63;
  const int s = scan_arena();
  const uint32_t nk = counts_before(sa, b, k, v.A);
  const uint64_t ns = static_cast<uint32_t>(__shfl(static_cast<int>(nk), s, 64));
  if (scan_rank() == 0 && threadIdx.x == 0) sa.nb[(static_cast<int64_t>(b) * sa.nstride + k) * NA + s] = static_cast<uint32_t>(ns);
  __shared__ uint32_t arena_n[NA];
  if (threadIdx.x < NA) arena_n[threadIdx.x] = nk;
  __syncthreads();
  unsigned long long* wst =
      sa.ws + (static_cast<int64_t>(b) * sa.nws + (blockIdx.x * (BLK / 64) + (threadIdx.x >> 6))) * WSTAT;
  const unsigned long long wold = lane < WSTAT ? wst[lane] : 0ull;
  const FacMask f1 = fac[k - 1], f2 = fac[k];
  const Trig t1 = trig[b * ld + k - 1], t2 = trig[b * ld + k];
  const T sn1 = static_cast<T>(t1.s), cm1a = static_cast<T>(t1.cm1);
  const T sn2 = static_cast<T>(t2.s), cm1b = static_cast<T>(t2.cm1);
  const uint64_t m1 = f1.occ | f1.vir, m2 = f2.occ | f2.vir;
  const uint32_t K1 = static_cast<uint32_t>(k), K2 = K1 + 1u;
  const uint64_t mask = v.H - 1;
  // c[1] visits, c[2] pairs, c[3] creates, c[5] new entries, c[6] pairs whose partner existed
  // c1a / c1b: visits of step k / k+1 (c1 of the statistics is their sum)
  unsigned long long c1a = 0, c1b = 0, c2 = 0, c3 = 0, c5 = 0, c6 = 0;
  unsigned int flags = 0;

  const uint64_t ebase = s * v.A;
  const uint64_t stride = scan_blocks() * BLK;
  uint64_t j = scan_rank() * BLK + threadIdx.x;
  for (uint64_t jw = scan_rank() * BLK + (threadIdx.x & ~63u); jw < ns; jw += stride, j += stride) {
    // this lane's work for the round; new entries are claimed by the whole
    // wave at its end
    bool want[4] = {false, false, false, false};
    uint64_t wfree[4] = {0, 0, 0, 0};
    T wamp[4];
    uint32_t wborn[4] = {0, 0, 0, 0};
    Quad Q;
    Q.q[0] = Q.q[1] = Q.q[2] = Q.q[3] = 0;
    do {
      if (j >= ns) break;
      const Slot<T> me = v.sl[ebase + j];
      const uint32_t m = me.meta;
      if ((m & DEAD) || (m & TAG) == K1 || (m & TAG) == K2) break;  // dead, or revived by this launch
      Q = make_quad(me.key, m1, m2, f1, f2);
      if (Q.comp == 1u) {  // acted on by neither factor
        c1a += 1;
        c1b += 1;
        break;
      }
      uint64_t ent[4], ff[4];
      bool pres[4], found[4];
      T a[4];
      ent[0] = ebase + j;
      pres[0] = found[0] = true;
      a[0] = me.amp;
      bool owner = true;
      // the first PH index slots from the home of every other member, loaded
      // together: most probes end inside them
      uint64_t home[4];
      Idx hv[4][PH];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        home[q] = home_slot(Q.q[q], v.H);
        if (Q.comp & (1u << q))
#pragma unroll
          for (int i = 0; i < PH; ++i) hv[q][i] = v.ix[(home[q] + i) & mask];
      }
      uint32_t pid[4];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        ent[q] = 0;
        ff[q] = v.H;
        pres[q] = found[q] = false;
        a[q] = T(0);
        pid[q] = NO_ID;
        if (!(Q.comp & (1u << q))) continue;
        Idx iv;
        if (find_slot_pre<PH>(v.ix, v.H, Q.q[q], home[q], hv[q], &ff[q], &iv) < 0) continue;
        found[q] = true;
        pid[q] = iv.id;
      }
      // entries of the members that existed when the launch began, loaded together
      Slot<T> pv[4];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        if (!found[q]) continue;
        if (pid[q] == NO_ID || created_here(pid[q], arena_n)) {  // created by this launch: not present
          found[q] = false;
          continue;
        }
        ent[q] = v.off(pid[q]);
        pv[q] = v.sl[ent[q]];
      }
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        if (!found[q]) continue;
        const uint32_t pt = pv[q].meta & TAG;
        // present when the launch started: alive and not revived by it
        pres[q] = !(pv[q].meta & DEAD) && pt != K1 && pt != K2;
        a[q] = pv[q].amp;
        if (pres[q] && Q.q[q] < Q.q[0]) owner = false;
      }
      if (!owner) break;
      bool exist[4];
      uint32_t born[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        exist[q] = pres[q];
        born[q] = 0u;
        if (!pres[q]) a[q] = T(0);
      }
      // one pair rotation of factor f on members u, w (absent members count as 0)
      auto rot = [&](int u, int w, const FacMask& f, T sn, T cm1, uint32_t Kt) {
        if (!pres[u] && !pres[w]) return;
        const int L = side(Q.q[u], f) == 1 ? u : w;
        const int U = L == u ? w : u;
        c2 += 1;
        if (pres[L] && pres[U]) c6 += 1;
        const T ss = (__popcll(Q.q[L] & f.sgn) & 1) ? -sn : sn;
        const T x = a[L], y = a[U];
        const T xn = x + fmaT<T>(x, cm1, -ss * y);
        const T yn = y + fmaT<T>(y, cm1, ss * x);
        a[L] = xn;
        a[U] = yn;
        if (!pres[L]) {
          pres[L] = true;
          born[L] = Kt;
          c3 += 1;
        }
        if (!pres[U]) {
          pres[U] = true;
          born[U] = Kt;
          c3 += 1;
        }
      };
      c1a += static_cast<unsigned long long>(pres[0]) + pres[1] + pres[2] + pres[3];
      if (Q.e1a) rot(0, 1, f1, sn1, cm1a, K1);
      if (Q.e1b && (Q.comp & 4u)) rot(2, 3, f1, sn1, cm1a, K1);
      c1b += static_cast<unsigned long long>(pres[0]) + pres[1] + pres[2] + pres[3];
      if (Q.e2a) rot(0, 2, f2, sn2, cm1b, K2);
      if (Q.e2b && (Q.comp & 2u)) rot(1, 3, f2, sn2, cm1b, K2);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (!pres[q]) continue;
        if (exist[q]) {
          v.sl[ent[q]].amp = a[q];
          continue;
        }
        if (found[q]) {  // a dead entry of an earlier sweep is revived in place
          v.sl[ent[q]].amp = a[q];
          v.born(ent[q]) = born[q];
          v.sl[ent[q]].meta = born[q];
          continue;
        }
        want[q] = true;
        wamp[q] = a[q];
        wborn[q] = born[q];
        wfree[q] = ff[q];
      }
    } while (false);
    uint64_t pos[4];
    const int ar = claim_positions<4>(sa, b, k, nk, want, pos);
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      if (!want[q]) continue;
      if (pos[q] >= v.A) {
        flags |= F_TABLE_FULL;
        continue;
      }
      const uint64_t e = ar * v.A + pos[q];
      v.sl[e].key = Q.q[q];
      v.sl[e].amp = wamp[q];
      v.sl[e].meta = wborn[q];
      v.born(e) = wborn[q];
      v.lam(e) = T(0);
      if (!index_insert(v.ix, v.H, Q.q[q], wfree[q], entry_id(ar, pos[q]))) {
        flags |= F_TABLE_FULL;
        continue;
      }
      c5 += 1;
    }
  }
  if (flags) atomicOr(&cnt[b].flags, flags);
  const unsigned int w1a = wave_u32(static_cast<unsigned int>(c1a)), w1b = wave_u32(static_cast<unsigned int>(c1b));
  const unsigned int w1 = w1a + w1b, w2 = wave_u32(static_cast<unsigned int>(c2));
  unsigned int w3 = wave_u32(static_cast<unsigned int>(c3)), w5 = wave_u32(static_cast<unsigned int>(c5));
  unsigned int w6 = wave_u32(static_cast<unsigned int>(c6));
  const int wsh = (blockIdx.x * (BLK / 64) + (threadIdx.x >> 6)) & (SH - 1);
  if (sa.pvis && lane == 0) {
    if (w1a) atomicAdd(&sa.pvis[sidx(sa, b, wsh, k)], w1a);
    if (w1b) atomicAdd(&sa.pvis[sidx(sa, b, wsh, k + 1)], w1b);
  }
  if (lane < 7) {
    const unsigned int mine = lane == 1 ? w1 : lane == 2 ? w2 : lane == 3 ? w3 : lane == 5 ? w5 : lane == 6 ? w6 : 0u;
    wst[lane] = wold + mine;
  }
}

// Reverse of steps k+1 then k (threshold 0: nothing was truncated, so the
// members present after the forward step are the alive ones; members created
// by a step are removed when it is undone).
template <class T, int PH>
__global__ __launch_bounds__(BLK) void k_rev2(Tab t, const FacMask* __restrict__ fac, const Trig* __restrict__ trig,
                                              int64_t ld, StepArr sa, Counters* cnt, int k) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int s = scan_arena();
  const uint64_t ns = static_cast<uint32_t>(__shfl(static_cast<int>(counts_reverse(sa, b, k + 1, v.A)), s, 64));
  const FacMask f1 = fac[k - 1], f2 = fac[k];
  const Trig t1 = trig[b * ld + k - 1], t2 = trig[b * ld + k];
  const T c1 = static_cast<T>(t1.c), sn1 = static_cast<T>(t1.s), cm1a = static_cast<T>(t1.cm1);
  const T c2 = static_cast<T>(t2.c), sn2 = static_cast<T>(t2.s), cm1b = static_cast<T>(t2.cm1);
  const uint64_t m1 = f1.occ | f1.vir, m2 = f2.occ | f2.vir;
  const uint32_t K1 = static_cast<uint32_t>(k), K2 = K1 + 1u;
  const uint64_t mask = v.H - 1;
  Fx g1 = fx_zero(), g2 = fx_zero();
  unsigned int flags = 0;

  const uint64_t ebase = s * v.A;
  const uint64_t stride = scan_blocks() * BLK;
  for (uint64_t j = scan_rank() * BLK + threadIdx.x; j < ns; j += stride) {
    const Slot<T> me = v.sl[ebase + j];
    const T lam_me = v.lam_pre(ebase + j);
    if (me.meta & DEAD) continue;
    const Quad Q = make_quad(me.key, m1, m2, f1, f2);
    if (Q.comp == 1u) continue;
    uint64_t ent[4];
    bool pres[4], found[4];
    uint32_t born[4];
    T a[4], l[4];
    ent[0] = ebase + j;
    pres[0] = found[0] = true;
    a[0] = me.amp;
    l[0] = v.lam_fin(me, lam_me);
    born[0] = me.meta & TAG;
    bool owner = true;
    // the first PH index slots from the home of every other member, loaded together
    uint64_t home[4];
    Idx hv[4][PH];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      home[q] = home_slot(Q.q[q], v.H);
      if (Q.comp & (1u << q))
#pragma unroll
        for (int i = 0; i < PH; ++i) hv[q][i] = v.ix[(home[q] + i) & mask];
    }
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      ent[q] = 0;
      pres[q] = found[q] = false;
      a[q] = T(0);
      l[q] = T(0);
      born[q] = 0u;
      if (!(Q.comp & (1u << q))) continue;
      uint64_t ff = v.H;
      Idx iv;
      if (find_slot_pre<PH>(v.ix, v.H, Q.q[q], home[q], hv[q], &ff, &iv) < 0) continue;
      if (iv.id == NO_ID) {
        flags |= F_INCONSISTENT;
        continue;
      }
      found[q] = true;
      ent[q] = v.off(iv.id);
    }
    // the members' entries (and adjoint values), loaded together
    Slot<T> pv[4];
    T pl[4];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      if (!found[q]) continue;
      pv[q] = v.sl[ent[q]];
      pl[q] = v.lam_pre(ent[q]);
    }
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      if (!found[q]) continue;
      const uint32_t pt = pv[q].meta & TAG;
      // present when the launch started: alive, or removed by this launch
      pres[q] = !(pv[q].meta & DEAD) || pt == K1 || pt == K2;
      if (!pres[q]) continue;
      if (Q.q[q] < Q.q[0]) owner = false;
      a[q] = pv[q].amp;
      l[q] = v.lam_fin(pv[q], pl[q]);
      born[q] = (pv[q].meta & DEAD) ? v.born(ent[q]) : pt;
    }
    if (!owner) continue;
    bool exist[4];
    uint32_t gone[4];  // step whose undo removed the member (0: kept)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      exist[q] = pres[q];
      gone[q] = 0u;
    }
    auto unrot = [&](int u, int w, const FacMask& f, T c, T sn, T cm1, uint32_t Kt, Fx& g) {
      if (!pres[u] && !pres[w]) return;
      const int L = side(Q.q[u], f) == 1 ? u : w;
      const int U = L == u ? w : u;
      const T ss = (__popcll(Q.q[L] & f.sgn) & 1) ? -sn : sn;
      const T lL = pres[L] ? l[L] : T(0), lU = pres[U] ? l[U] : T(0);
      const T xp = pres[L] ? a[L] : T(0), yp = pres[U] ? a[U] : T(0);
      const T wL = lL + fmaT<T>(lL, cm1, ss * lU);
      const T wU = lU + fmaT<T>(lU, cm1, -ss * lL);
      T x, y;
      if (pres[L] && pres[U]) {
        x = xp + fmaT<T>(xp, cm1, ss * yp);
        y = yp + fmaT<T>(yp, cm1, -ss * xp);
      } else if (pres[L]) {
        x = xp / c;
        y = T(0);
      } else {
        x = T(0);
        y = yp / c;
      }
      const double sgn = (__popcll(Q.q[L] & f.sgn) & 1) ? -1.0 : 1.0;
      g = fx_add(g, fx_from(sgn * (static_cast<double>(wU) * static_cast<double>(x) -
                                   static_cast<double>(wL) * static_cast<double>(y))));
      const bool hL = pres[L], hU = pres[U];
      if (hL) {
        if (born[L] == Kt) {
          if (!hU) flags |= F_INCONSISTENT;
          pres[L] = false;
          gone[L] = Kt;
        } else {
          a[L] = x;
          l[L] = wL;
        }
      }
      if (hU) {
        if (born[U] == Kt) {
          if (!hL) flags |= F_INCONSISTENT;
          pres[U] = false;
          gone[U] = Kt;
        } else {
          a[U] = y;
          l[U] = wU;
        }
      }
    };
    if (Q.e2a) unrot(0, 2, f2, c2, sn2, cm1b, K2, g2);
    if (Q.e2b && (Q.comp & 2u)) unrot(1, 3, f2, c2, sn2, cm1b, K2, g2);
    if (Q.e1a) unrot(0, 1, f1, c1, sn1, cm1a, K1, g1);
    if (Q.e1b && (Q.comp & 4u)) unrot(2, 3, f1, c1, sn1, cm1a, K1, g1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!exist[q]) continue;
      const uint64_t d = ent[q];
      if (gone[q]) {
        v.sl[d].meta = DEAD | gone[q];
      } else {
        v.sl[d].amp = a[q];
        v.lam(d) = l[q];
        v.sl[d].meta = born[q];
      }
    }
  }
  if (flags) atomicOr(&cnt[b].flags, flags);
  const Fx w1 = wave_fx(g1), w2 = wave_fx(g2);
  const int wsh = (blockIdx.x * (BLK / 64) + (threadIdx.x >> 6)) & (SH - 1);
  if ((threadIdx.x & 63) == 0) {
    if (fx_nonzero(w1)) fx3_atomic_add(&sa.gacc[sidx(sa, b, wsh, k)], w1);
    if (fx_nonzero(w2)) fx3_atomic_add(&sa.gacc[sidx(sa, b, wsh, k + 1)], w2);
  }
}

template <class T>
__global__ void k_log_restore(Tab t, LogArr lg, StepArr sa, int k) {
  restore_step<T>(t, lg, sa, k);
}

// ---------------------------------------------------------------------------
// persistent sweeps: one cooperative launch runs many steps
// ---------------------------------------------------------------------------
// Grid-wide barrier of a cooperative (all blocks co-resident) launch.
// Arrivals are counted monotonically: barrier e completes when the counter
// reaches e * nblocks.  Agent-scope fences publish each step's writes to all
// XCDs before the next step reads them.  Every wait is bounded; when the
// bound is hit the sticky timeout flag is raised, later barriers return at
// once and the host reports an error, so the launch always terminates.
constexpr unsigned int SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ void grid_barrier(Sync* sy, unsigned int target) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(&sy->count, 1u);
    for (unsigned int it = 0;; ++it) {
      if (__hip_atomic_load(&sy->count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(&sy->timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
      if (it >= SPIN_LIMIT) {
        atomicOr(&sy->timeout, 1u);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
  }
  __syncthreads();
}

// A sweep may take several cooperative launches (one per checkpoint
// interval): the barrier count restarts for each, the timeout flag only at the
// start of the sweep, so a timeout in any launch is still reported at its end.
__global__ void k_sync_reset(Sync* sy, int clear_timeout) {
  if (threadIdx.x == 0) {
    sy->count = 0u;
    if (clear_timeout) sy->timeout = 0u;
  }
}

// forward steps k0..k1 (inclusive)
template <class T>
__global__ __launch_bounds__(BLK) void k_fwd_sweep(Tab t, const FacMask* __restrict__ fac,
                                                   const Trig* __restrict__ trig, int64_t ld, StepArr sa,
                                                   Counters* cnt, LogArr lg, int k0, int k1, double thr,
                                                   int prune_first, int log_on, Sync* sy) {
  const unsigned int nblk = gridDim.x * gridDim.y;
  unsigned int epoch = 0;
  for (int k = k0; k <= k1; ++k) {
    if (sa.ea)
      fwd_step<T, true>(t, fac, trig, ld, sa, cnt, lg, k, thr, prune_first && k == k0, log_on, NO_LIMIT, 0,
                        static_cast<int>(gridDim.y));
    else
      fwd_step<T, false>(t, fac, trig, ld, sa, cnt, lg, k, thr, prune_first && k == k0, log_on, NO_LIMIT, 0,
                         static_cast<int>(gridDim.y));
    grid_barrier(sy, ++epoch * nblk);
  }
}

// reverse steps k_hi down to k_lo, with the log restores of the steps whose
// forward pass overwrote dead entries (rmax[k] > 0)
template <class T>
__global__ __launch_bounds__(BLK) void k_rev_sweep(Tab t, const FacMask* __restrict__ fac,
                                                   const Trig* __restrict__ trig, int64_t ld, StepArr sa,
                                                   Counters* cnt, LogArr lg, int k_hi, int k_lo, Sync* sy) {
  const unsigned int nblk = gridDim.x * gridDim.y;
  unsigned int epoch = 0;
  for (int k = k_hi; k >= k_lo; --k) {
    rev_step<T>(t, fac, trig, ld, sa, cnt, k, 0);
    grid_barrier(sy, ++epoch * nblk);
    if (sa.rmax[k]) {
      restore_step<T>(t, lg, sa, k);
      grid_barrier(sy, ++epoch * nblk);
    }
  }
}


// ---------------------------------------------------------------------------
// energy: compact live entries, sigma = H psi on the support, E
// ---------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(BLK) void k_compact(Tab t, Compact cp, Counters* cnt) {
  // one counter claim per block and pass (the waves' counts combined in LDS),
  // not per wave: the claims all go to one address
  __shared__ unsigned int wcount[BLK / 64];
  __shared__ unsigned long long wbase[BLK / 64];
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int a = scan_arena();
  const uint64_t n = t.ac[b * NA + a];
  const uint64_t stride = scan_blocks() * BLK;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (uint64_t j0 = scan_rank() * BLK; j0 < n; j0 += stride) {  // the same passes for the whole block
    const uint64_t j = j0 + threadIdx.x;
    bool live = false;
    Slot<T> me;
    me.key = 0;
    me.amp = T(0);
    if (j < n) {
      me = v.sl[a * v.A + j];
      live = !(me.meta & DEAD);
    }
    const unsigned long long mask = __ballot(live);
    if (lane == 0) wcount[w] = static_cast<unsigned int>(__popcll(mask));
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long tot = 0;
      for (int i = 0; i < BLK / 64; ++i) tot += wcount[i];
      unsigned long long basep = tot ? atomicAdd(&cnt[b].ncompact, tot) : 0ull;
      for (int i = 0; i < BLK / 64; ++i) {
        wbase[i] = basep;
        basep += wcount[i];
      }
    }
    __syncthreads();
    const unsigned long long basep = wbase[w];
    __syncthreads();  // wcount / wbase are rewritten by the next pass
    if (live) {
      const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
      const uint64_t pos = basep + __popcll(below);
      cp.key[b * cp.cs + pos] = me.key;
      cp.amp[b * cp.cs + pos] = static_cast<double>(me.amp);
      cp.slot[b * cp.cs + pos] = entry_id(a, j);
      cp.sig[b * cp.cs + pos] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// checkpoints: a snapshot of the live (key, raw amplitude) pairs after a
// forward step; the reverse sweep writes it back over the amplitudes it has
// reconstructed for the same step, so the rounding drift of inverted steps
// spans at most one checkpoint interval.  The support is reconstructed
// exactly, so every snapshot key is alive at that point.
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(BLK) void k_snapshot(Tab t, StepArr sa, Snap sn, int k) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int a = scan_arena();
  const uint64_t n = static_cast<uint32_t>(__shfl(static_cast<int>(counts_after(sa, b, k, v.A)), a, 64));
  const uint64_t stride = scan_blocks() * BLK;
  const int lane = threadIdx.x & 63;
  T* amp = static_cast<T*>(sn.amp);
  for (uint64_t j0 = scan_rank() * BLK + (threadIdx.x & ~63u); j0 < n; j0 += stride) {  // uniform per wave
    const uint64_t j = j0 + lane;
    bool live = false;
    Slot<T> me;
    me.key = 0;
    me.amp = T(0);
    if (j < n) {
      me = v.sl[a * v.A + j];
      live = !(me.meta & DEAD);
    }
    const unsigned long long mask = __ballot(live);
    if (!mask) continue;
    const int leader = __ffsll(static_cast<long long>(mask)) - 1;
    unsigned long long basep = 0;
    if (lane == leader) basep = atomicAdd(&sn.count[b], static_cast<unsigned long long>(__popcll(mask)));
    basep = __shfl(basep, leader, 64);
    if (live) {
      const unsigned long long below = lane ? (mask & ((1ull << lane) - 1ull)) : 0ull;
      const uint64_t pos = basep + __popcll(below);
      if (pos < sn.cap) {
        sn.key[b * sn.cap + pos] = me.key;
        amp[b * sn.cap + pos] = me.amp;
      }
    }
  }
}

template <class T>
__global__ __launch_bounds__(BLK) void k_snap_restore(Tab t, Snap sn, Counters* cnt) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const uint64_t n = sn.count[b] < sn.cap ? sn.count[b] : sn.cap;
  const T* amp = static_cast<const T*>(sn.amp);
  for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint64_t ff = v.H;
    Idx iv;
    if (find_slot(v.ix, v.H, sn.key[b * sn.cap + i], &ff, &iv) < 0 || iv.id == NO_ID ||
        (v.sl[v.off(iv.id)].meta & DEAD)) {
      atomicOr(&cnt[b].flags, F_INCONSISTENT);
      continue;
    }
    v.sl[v.off(iv.id)].amp = amp[b * sn.cap + i];
  }
}

// entropy of the state (alive entries) into step k's sums
template <class T>
__global__ __launch_bounds__(BLK) void k_entropy_scan(Tab t, StepArr sa, int k) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int a = scan_arena();
  const uint64_t n = t.ac[b * NA + a];
  Fx ea = fx_zero(), eb = fx_zero();
  for (uint64_t j = scan_rank() * BLK + threadIdx.x; j < n; j += scan_blocks() * BLK) {
    const Slot<T> x = v.sl[a * v.A + j];
    if (!(x.meta & DEAD)) ent_add(ea, eb, static_cast<double>(x.amp));
  }
  ent_flush(sa, b, k, ea, eb);
}

// Entropy (Eq. 6) after step k from the exact sums A = sum r^2 ln r^2 and
// B = sum r^2 of the raw amplitudes: with p = r^2 / B, -sum p ln p = ln B - A / B.
__global__ void k_entropy_final(StepArr sa, int64_t M) {
  const int b = blockIdx.y;
  for (int64_t k = blockIdx.x * blockDim.x + threadIdx.x; k <= M; k += gridDim.x * blockDim.x) {
    Fx A = fx_zero(), Bs = fx_zero();
    for (int q = 0; q < ES; ++q) {
      const int64_t idx = (static_cast<int64_t>(b) * ES + q) * sa.stride + k;
      A = fx_add(A, fx3_value(sa.ea[idx]));
      Bs = fx_add(Bs, fx3_value(sa.eb[idx]));
    }
    const double a = fx_to_d(A), bb = fx_to_d(Bs);
    sa.ent[static_cast<int64_t>(b) * sa.stride + k] = bb > 0.0 ? log(bb) - a / bb : 0.0;
  }
}

// ---------------------------------------------------------------------------
// N_MAX / N_CUT truncation (Methods section): when more than N_MAX entries
// are live after step k, keep the N_CUT of largest rank (|c|, then smaller
// determinant) and remove the rest like a threshold cut (tombstone with the
// pre-truncation amplitude, removed weight into step k's renormalisation).
// The N_CUT-th rank is found by a radix selection, TK_BITS per pass from the
// top: each pass histograms the digit of the entries that match the digits
// chosen so far, and one block picks the digit holding the boundary.
// ---------------------------------------------------------------------------
struct R128 {
  unsigned long long hi, lo;
};

__device__ __forceinline__ R128 shr128(R128 r, int s) {
  if (s <= 0) return r;
  if (s >= 128) return R128{0ull, 0ull};
  if (s >= 64) return R128{0ull, r.hi >> (s - 64)};
  return R128{r.hi >> s, (r.lo >> s) | (r.hi << (64 - s))};
}

__device__ __forceinline__ bool lt128(R128 a, R128 b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

template <class T>
__device__ __forceinline__ R128 rank_of(uint64_t key, T amp);
template <>
__device__ __forceinline__ R128 rank_of<float>(uint64_t key, float amp) {
  return R128{static_cast<unsigned long long>(__float_as_uint(fabsf(amp))), ~key};
}
template <>
__device__ __forceinline__ R128 rank_of<double>(uint64_t key, double amp) {
  return R128{static_cast<unsigned long long>(__double_as_longlong(fabs(amp))), ~key};
}
template <class T>
constexpr int rank_bits() {
  return sizeof(T) == 4 ? 96 : 128;
}

// digit of pass p: bits [top - w, top) with top = nbits - TK_BITS p
__device__ __forceinline__ unsigned digit_of(R128 r, int nbits, int pass) {
  const int top = nbits - TK_BITS * pass;
  const int low = top > TK_BITS ? top - TK_BITS : 0;
  return static_cast<unsigned>(shr128(r, low).lo) & ((1u << (top - low)) - 1u);
}

// The selection of pass `pass` from its histogram, made by a whole block
// (every block of the launch that follows the pass computes the same result):
// in = the state after the previous pass's selection (unused for pass 0).
template <class T>
__device__ TKState tk_select(const unsigned int* __restrict__ hist, const TKState* in, int pass,
                             unsigned long long n_max, unsigned long long n_cut) {
  constexpr int nbits = rank_bits<T>();
  constexpr int PER = TK_BINS / BLK;
  __shared__ unsigned long long part[BLK];
  __shared__ TKState out;
  unsigned long long my = 0;
  for (int j = 0; j < PER; ++j) my += hist[TK_BINS - 1 - (threadIdx.x * PER + j)];
  part[threadIdx.x] = my;
  __syncthreads();
  if (threadIdx.x == 0) {
    TKState o;
    bool go = true;
    if (pass == 0) {
      unsigned long long total = 0;
      for (int i = 0; i < BLK; ++i) total += part[i];
      o.pre_hi = o.pre_lo = 0ull;
      o.depth = 0;
      o.done = 0;
      o.nokill = 0;
      o.pad = 0;
      o.remaining = n_cut;
      if (total <= n_max) {
        o.done = 1;
        o.nokill = 1;
        go = false;
      }
    } else {
      o = *in;
      if (o.done) go = false;
    }
    if (go) {
      const unsigned long long rem = o.remaining;
      unsigned long long cum = 0;  // entries of higher digits
      int i = 0;
      while (i < BLK - 1 && cum + part[i] < rem) cum += part[i++];
      int d = TK_BINS - 1 - i * PER;
      for (int j = 0; j < PER; ++j) {
        d = TK_BINS - 1 - (i * PER + j);
        const unsigned long long hd = hist[d];
        if (cum + hd >= rem) break;
        cum += hd;
      }
      const unsigned long long need = rem - cum;  // to keep inside digit d
      const int top = nbits - TK_BITS * pass;
      const int w = top > TK_BITS ? TK_BITS : top;
      // prefix = (prefix << w) | d
      R128 pre{o.pre_hi, o.pre_lo};
      pre = R128{(pre.hi << w) | (pre.lo >> (64 - w)), (pre.lo << w) | static_cast<unsigned long long>(d)};
      o.pre_hi = pre.hi;
      o.pre_lo = pre.lo;
      o.depth = pass + 1;
      o.remaining = need;
      if (hist[d] == need || top <= TK_BITS) o.done = 1;
    }
    out = o;
  }
  __syncthreads();
  return out;
}

// Pass `pass` of the selection: the previous pass's selection (every block),
// then, unless it finished, the histogram of this pass's digit over the
// entries that match the digits chosen so far.  Also clears the histogram
// buffer the next pass fills.
template <class T>
__global__ __launch_bounds__(BLK) void k_topk_pass(Tab t, StepArr sa, TopK* tk, const Counters* cnt, int k, int pass,
                                                    unsigned long long n_max, unsigned long long n_cut) {
  const int b = blockIdx.y;
  if (static_cast<uint32_t>(k) >= cnt[0].stop) return;
  TopK& tb = tk[b];
  constexpr int nbits = rank_bits<T>();
  TKState st{};
  if (pass > 0) {
    st = tk_select<T>(tb.hist[(pass - 1) % 3], &tb.st[pass & 1], pass - 1, n_max, n_cut);
    if (blockIdx.x == 0 && threadIdx.x == 0) tb.st[(pass - 1) & 1] = st;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < TK_BINS; i += gridDim.x * blockDim.x)
    tb.hist[(pass + 1) % 3][i] = 0u;
  if (pass > 0 && st.done) return;
  __shared__ unsigned int h[TK_BINS];
  for (int i = threadIdx.x; i < TK_BINS; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const R128 pre{st.pre_hi, st.pre_lo};
  const int shift = nbits - TK_BITS * pass;
  const View<T> v = view<T>(t, b);
  const int a = scan_arena();
  const uint64_t n = static_cast<uint32_t>(__shfl(static_cast<int>(counts_after(sa, b, k, v.A)), a, 64));
  for (uint64_t j = scan_rank() * BLK + threadIdx.x; j < n; j += scan_blocks() * BLK) {
    const Slot<T> x = v.sl[a * v.A + j];
    if (x.meta & DEAD) continue;
    const R128 r = rank_of<T>(x.key, x.amp);
    if (pass > 0) {
      const R128 top = shr128(r, shift);
      if (top.hi != pre.hi || top.lo != pre.lo) continue;
    }
    atomicAdd(&h[digit_of(r, nbits, pass)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < TK_BINS; i += blockDim.x)
    if (h[i]) atomicAdd(&tb.hist[pass % 3][i], h[i]);
}

template <class T>
__global__ __launch_bounds__(BLK) void k_topk_kill(Tab t, StepArr sa, Counters* cnt, TopK* tk, int k,
                                                    unsigned long long n_max, unsigned long long n_cut) {
  const int b = blockIdx.y;
  if (static_cast<uint32_t>(k) >= cnt[0].stop) return;
  constexpr int nbits = rank_bits<T>();
  constexpr int npass = (nbits + TK_BITS - 1) / TK_BITS;
  // the first pass of the next selection fills hist[0]: the one this
  // selection filled at pass npass - 2 is cleared here
  static_assert(npass % 3 == 2, "the histogram buffers rotate back to hist[0]");
  TopK& tb = tk[b];
  const TKState st = tk_select<T>(tb.hist[(npass - 1) % 3], &tb.st[npass & 1], npass - 1, n_max, n_cut);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < TK_BINS; i += gridDim.x * blockDim.x)
    tb.hist[(npass - 2) % 3][i] = 0u;
  if (st.nokill || st.depth == 0) return;
  const int sel = TK_BITS * st.depth < nbits ? TK_BITS * st.depth : nbits;
  const R128 pre{st.pre_hi, st.pre_lo};
  const View<T> v = view<T>(t, b);
  const uint32_t K = static_cast<uint32_t>(k);
  const int a = scan_arena();
  const uint64_t n = static_cast<uint32_t>(__shfl(static_cast<int>(counts_after(sa, b, k, v.A)), a, 64));
  Fx w = fx_zero(), ea = fx_zero(), eb = fx_zero();
  unsigned int nk = 0;
  for (uint64_t j = scan_rank() * BLK + threadIdx.x; j < n; j += scan_blocks() * BLK) {
    const uint64_t e = a * v.A + j;
    const Slot<T> x = v.sl[e];
    if (x.meta & DEAD) continue;
    if (!lt128(shr128(rank_of<T>(x.key, x.amp), nbits - sel), pre)) continue;
    v.sl[e].meta = DEAD | K;  // the entry keeps the pre-truncation amplitude
    const double r = static_cast<double>(x.amp);
    w = fx_add(w, fx_from(r * r));
    ++nk;
    if (sa.ea) ent_add(ea, eb, r);
  }
  const unsigned int c = wave_u32(nk);
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * (BLK / 64) + (threadIdx.x >> 6);
  if (c) {
    const Fx ws = wave_fx(w);
    if (lane == 0) {
      fx3_atomic_add(&sa.pw[sidx(sa, b, wv & (SH - 1), k)], ws);
      atomicAdd(&sa.pcnt[sidx(sa, b, wv & (SH - 1), k)], c);
    }
    if (sa.ea) {  // removed entries leave the entropy sums
      ea = wave_fx(ea);
      eb = wave_fx(eb);
      if (lane == 0) {
        const int64_t idx = (static_cast<int64_t>(b) * ES + (wv & (ES - 1))) * sa.stride + k;
        fx3_atomic_add(&sa.ea[idx], Fx{~ea.lo + 1ull, ~ea.hi + (ea.lo == 0ull ? 1ull : 0ull)});
        fx3_atomic_add(&sa.eb[idx], Fx{~eb.lo + 1ull, ~eb.hi + (eb.lo == 0ull ? 1ull : 0ull)});
      }
    }
    // statistics: removed count (slot 0) and removals of live entries (slot 4)
    unsigned long long* wst = sa.ws + (static_cast<int64_t>(b) * sa.nws + wv) * WSTAT;
    if (lane == 0) wst[0] += c;
    if (lane == 4) wst[4] += c;
  }
}

__global__ void k_zero_u64(unsigned long long* p, uint64_t n) {
  for (uint64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

__device__ __forceinline__ uint64_t between(int lo, int hi) {  // bits lo+1 .. hi-1
  return ((1ull << hi) - 1ull) & ~((2ull << lo) - 1ull);
}

// (pq|rs) of the n^4 array.  n <= 32, so every partial index stays below
// 2^20 and the full-rate 24-bit multiplier computes it exactly.
__device__ __forceinline__ double eri(const double* __restrict__ h2, int n, int p, int q, int r, int s) {
  const unsigned int un = static_cast<unsigned int>(n);
  const unsigned int i = __umul24(__umul24(__umul24(static_cast<unsigned int>(p), un) + q, un) + r, un) + s;
  return h2[i];
}

// <I|J> parts of H by the Slater-Condon rules; C = the orbitals occupied in
// both, the sign from those strictly between the moved ones.
// Single: spin-orbital p of I replaced by q.
__device__ __forceinline__ double h_single(uint64_t C, int p, int q, const double* __restrict__ h1,
                                           const double* __restrict__ h2, int n) {
  if ((p ^ q) & 1) return 0.0;
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  const int P = p >> 1, Q = q >> 1, sp = p & 1;
  double v = h1[__umul24(static_cast<unsigned int>(P), static_cast<unsigned int>(n)) + Q];
  for (uint64_t mm = C; mm; mm &= mm - 1ull) {
    const int kk = __ffsll(static_cast<long long>(mm)) - 1;
    const int Kk = kk >> 1;
    v += eri(h2, n, P, Q, Kk, Kk);
    if ((kk & 1) == sp) v -= eri(h2, n, P, Kk, Kk, Q);
  }
  return (__popcll(C & between(lo, hi)) & 1) ? -v : v;
}

// Double: spin-orbitals p1 < p2 of I replaced by q1 < q2.
__device__ __forceinline__ double h_double(uint64_t C, int p1, int p2, int q1, int q2,
                                           const double* __restrict__ h2, int n) {
  double v = 0.0;
  if (((p1 ^ q1) & 1) == 0 && ((p2 ^ q2) & 1) == 0) v += eri(h2, n, p1 >> 1, q1 >> 1, p2 >> 1, q2 >> 1);
  if (((p1 ^ q2) & 1) == 0 && ((p2 ^ q1) & 1) == 0) v -= eri(h2, n, p1 >> 1, q2 >> 1, p2 >> 1, q1 >> 1);
  const int par = __popcll(C & between(q1, q2)) + __popcll(C & between(p1, p2));
  return (par & 1) ? -v : v;
}

// <I|H|J> for determinants differing in pc = 2 (single) or 4 (double) bits.
__device__ double h_offdiag(uint64_t I, uint64_t J, int pc, const double* __restrict__ h1,
                            const double* __restrict__ h2, int n) {
  const uint64_t d = I ^ J, C = I & J;
  if (pc == 2)
    return h_single(C, __ffsll(static_cast<long long>(I & d)) - 1, __ffsll(static_cast<long long>(J & d)) - 1, h1,
                    h2, n);
  const uint64_t dI = I & d, dJ = J & d;
  return h_double(C, __ffsll(static_cast<long long>(dI)) - 1, 63 - __clzll(static_cast<long long>(dI)),
                  __ffsll(static_cast<long long>(dJ)) - 1, 63 - __clzll(static_cast<long long>(dJ)), h2, n);
}

// <I|H|I> from the one-electron diagonal d1[P] = h_PP and the Coulomb and
// exchange tables J[P][Q] = (PP|QQ), K[P][Q] = (PQ|QP) staged in LDS (the
// same terms, added in the same order, as the n^4 integrals give them).
__device__ double h_diag(uint64_t I, const double* d1, const double* J, const double* K, int n) {
  double v = 0.0;
  for (uint64_t a = I; a; a &= a - 1ull) {
    const int p = __ffsll(static_cast<long long>(a)) - 1;
    const int P = p >> 1;
    const unsigned int row = __umul24(static_cast<unsigned int>(P), static_cast<unsigned int>(n));
    v += d1[P];
    for (uint64_t bb = a & (a - 1ull); bb; bb &= bb - 1ull) {
      const int q = __ffsll(static_cast<long long>(bb)) - 1;
      const int Q = q >> 1;
      v += J[row + Q];
      if (((p ^ q) & 1) == 0) v -= K[row + Q];
    }
  }
  return v;
}

constexpr int SG = 16;               // lanes per determinant in the sigma kernel
constexpr int SGU = 4;               // excitations each lane probes together
constexpr int TRI = 32 * 31 / 2;     // index pairs i1 < i2 < 32
constexpr int LROW = 132;            // bytes per group of orbital lists (padded: no LDS bank conflicts)

// Orbital lists of one determinant: occupied alpha, occupied beta, empty
// alpha, empty beta (spin-orbital indices), in one LDS row.
struct Lists {
  const uint8_t* oa;
  const uint8_t* ob;
  const uint8_t* va;
  const uint8_t* vb;
  int nA, nB, mA, mB;  // occupied / empty counts per spin
  int sA, sB, dAA, dBB, dAB;  // sizes of the excitation classes
  int pA, pB;                 // empty-orbital pairs per spin
  float rmA, rmB, rnB, rpA, rpB;  // 1/mA, 1/mB, 1/nB, 1/pA, 1/pB (unused where the divisor is 0)
};

// a / d and a % d for a < 2^22 and 1 <= d < 2^10, with rd = 1/d correctly
// rounded to float: a * rd is within a/d * 2^-23 < 1/2 of a/d, so it
// truncates to the true quotient or one off, and one remainder test corrects
// it.  Full-rate instructions only (the integer divider's sequence uses
// quarter-rate ones).
__device__ __forceinline__ unsigned int udiv_small(unsigned int a, unsigned int d, float rd, unsigned int* rem) {
  unsigned int q = static_cast<unsigned int>(static_cast<float>(a) * rd);
  int r = static_cast<int>(a) - static_cast<int>(__umul24(q, d));
  if (r < 0) {
    --q;
    r += static_cast<int>(d);
  } else if (r >= static_cast<int>(d)) {
    ++q;
    r -= static_cast<int>(d);
  }
  *rem = static_cast<unsigned int>(r);
  return q;
}

// Excitation number e (0 <= e < total) of I: alpha singles, beta singles,
// alpha-alpha doubles, beta-beta doubles, alpha-beta doubles, each a flat
// range.  Returns J; *mv holds the moved spin-orbitals, one per byte: a
// single p -> q as p | q << 16, a double p1 < p2 -> q1 < q2 as
// p1 | p2 << 8 | q1 << 16 | q2 << 24; *rank is 2 (single) or 4 (double).
__device__ __forceinline__ uint64_t excite(uint64_t I, int e, const Lists& L, const uint16_t* tri, int* rank,
                                           unsigned int* mv) {
  unsigned int r;
  if (e < L.sA + L.sB) {
    const bool beta = e >= L.sA;
    if (beta) e -= L.sA;
    const unsigned int x = beta ? udiv_small(e, L.mB, L.rmB, &r) : udiv_small(e, L.mA, L.rmA, &r);
    const unsigned int p = beta ? L.ob[x] : L.oa[x], q = beta ? L.vb[r] : L.va[r];
    *rank = 2;
    *mv = p | q << 16;
    return I ^ (1ull << p) ^ (1ull << q);
  }
  e -= L.sA + L.sB;
  *rank = 4;
  unsigned int p1, p2, q1, q2;
  if (e < L.dAA + L.dBB) {
    const bool beta = e >= L.dAA;
    if (beta) e -= L.dAA;
    const uint8_t* oc = beta ? L.ob : L.oa;
    const uint8_t* vi = beta ? L.vb : L.va;
    const unsigned int x = udiv_small(e, beta ? L.pB : L.pA, beta ? L.rpB : L.rpA, &r);
    const uint16_t po = tri[x], pv = tri[r];
    // the lists ascend and tri pairs ascend: p1 < p2, q1 < q2
    p1 = oc[po & 255];
    p2 = oc[po >> 8];
    q1 = vi[pv & 255];
    q2 = vi[pv >> 8];
  } else {
    e -= L.dAA + L.dBB;
    unsigned int xa, xb, jb;
    const unsigned int ea = udiv_small(e, L.mA, L.rmA, &xa);
    const unsigned int eb = udiv_small(ea, L.mB, L.rmB, &xb);
    const unsigned int ia = udiv_small(eb, L.nB, L.rnB, &jb);
    const unsigned int oA = L.oa[ia], oB = L.ob[jb], vA = L.va[xa], vB = L.vb[xb];
    p1 = oA < oB ? oA : oB;
    p2 = oA < oB ? oB : oA;
    q1 = vA < vB ? vA : vB;
    q2 = vA < vB ? vB : vA;
  }
  *mv = p1 | p2 << 8 | q1 << 16 | q2 << 24;
  return I ^ (1ull << p1) ^ (1ull << p2) ^ (1ull << q1) ^ (1ull << q2);
}

// sigma_I = sum_J <I|H|J> c_J over the single and double excitations J of I
// that are alive in the state (off-diagonal part; the diagonal is added in
// k_energy_reduce).  SG lanes of one wave share I and its orbital lists (one
// LDS row per group, written identically by all its lanes before any of them
// reads it: a wave executes its LDS instructions in order).  The excitations
// of I form one flat index range; lane g takes g, g+SG, ..., SGU at a time,
// loading the home slots of the SGU determinants together before resolving
// the probes.  Each lane adds its terms in index order and the SG partial
// sums are combined by a fixed shuffle tree: sigma is bit-reproducible.
template <class T>
__global__ __launch_bounds__(BLK) void k_sigma(Tab t, Compact cp, const Counters* cnt,
                                               const double* __restrict__ h1, const double* __restrict__ h2,
                                               int nq, int singles_only) {
  __shared__ uint16_t tri[TRI];
  __shared__ uint8_t lists[(BLK / SG) * LROW];
  for (int e = threadIdx.x; e < TRI; e += blockDim.x) {
    int i2 = 1;
    while ((i2 + 1) * i2 / 2 <= e) ++i2;
    const int i1 = e - i2 * (i2 - 1) / 2;
    tri[e] = static_cast<uint16_t>(i1 | (i2 << 8));
  }
  __syncthreads();
  const int b = blockIdx.y;
  const uint64_t H = t.H;
  const int64_t N = static_cast<int64_t>(cnt[b].ncompact);
  const View<T> v = view<T>(t, b);
  const int n = nq / 2;
  const int g = threadIdx.x & (SG - 1);
  const uint64_t full = nq >= 64 ? ~0ull : ((1ull << nq) - 1ull);
  const uint64_t ALPHA = 0x5555555555555555ull & full, BETA = 0xAAAAAAAAAAAAAAAAull & full;
  const int64_t gstride = static_cast<int64_t>(gridDim.x) * (blockDim.x / SG);
  uint8_t* row = lists + (threadIdx.x / SG) * LROW;
  auto fill = [](uint8_t* dst, uint64_t m) -> int {
    int c = 0;
    for (; m; m &= m - 1ull) dst[c++] = static_cast<uint8_t>(__ffsll(static_cast<long long>(m)) - 1);
    return c;
  };
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / SG; i < N; i += gstride) {
    const uint64_t I = cp.key[b * cp.cs + i];
    Lists L;
    L.nA = fill(row, I & ALPHA);
    L.nB = fill(row + 32, I & BETA);
    L.mA = fill(row + 64, ~I & ALPHA);
    L.mB = fill(row + 96, ~I & BETA);
    L.oa = row;
    L.ob = row + 32;
    L.va = row + 64;
    L.vb = row + 96;
    L.sA = L.nA * L.mA;
    L.sB = L.nB * L.mB;
    L.pA = L.mA * (L.mA - 1) / 2;
    L.pB = L.mB * (L.mB - 1) / 2;
    L.dAA = L.nA * (L.nA - 1) / 2 * L.pA;
    L.dBB = L.nB * (L.nB - 1) / 2 * L.pB;
    L.dAB = L.nA * L.nB * L.mA * L.mB;
    L.rmA = __frcp_rn(static_cast<float>(L.mA));
    L.rmB = __frcp_rn(static_cast<float>(L.mB));
    L.rnB = __frcp_rn(static_cast<float>(L.nB));
    L.rpA = __frcp_rn(static_cast<float>(L.pA));
    L.rpB = __frcp_rn(static_cast<float>(L.pB));
    const int total = singles_only ? L.sA + L.sB : L.sA + L.sB + L.dAA + L.dBB + L.dAB;
    double acc = 0.0;
    for (int e0 = g; e0 < total; e0 += SG * SGU) {
      uint64_t J[SGU], home[SGU];
      int rank[SGU];
      unsigned int mv[SGU];
      Idx hv[SGU][4];
#pragma unroll
      for (int u = 0; u < SGU; ++u) {
        const int e = e0 + u * SG;
        if (e < total) {
          J[u] = excite(I, e, L, tri, &rank[u], &mv[u]);
          home[u] = home_slot(J[u], H);
#pragma unroll
          for (int q = 0; q < 4; ++q) hv[u][q] = v.ix[home[u] + q];
        }
      }
      // resolve the index probes, then load the entries found together
      uint64_t pe[SGU];
      bool hit[SGU];
#pragma unroll
      for (int u = 0; u < SGU; ++u) {
        hit[u] = false;
        if (e0 + u * SG >= total) continue;
        uint64_t ff;
        Idx iv;
        if (find_slot_pre<4>(v.ix, H, J[u], home[u], hv[u], &ff, &iv) >= 0 && iv.id != NO_ID) {
          hit[u] = true;
          pe[u] = v.off(iv.id);
        }
      }
      Slot<T> pv[SGU];
#pragma unroll
      for (int u = 0; u < SGU; ++u)
        if (hit[u]) pv[u] = v.sl[pe[u]];
#pragma unroll
      for (int u = 0; u < SGU; ++u) {
        if (!hit[u] || (pv[u].meta & DEAD)) continue;
        const uint64_t C = I & J[u];
        const unsigned int m = mv[u];
        const double h = rank[u] == 2 ? h_single(C, m & 255, (m >> 16) & 255, h1, h2, n)
                                      : h_double(C, m & 255, (m >> 8) & 255, (m >> 16) & 255, m >> 24, h2, n);
        acc += h * static_cast<double>(pv[u].amp);
      }
    }
#pragma unroll
    for (int o = SG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, SG);
    if (g == 0) cp.sig[b * cp.cs + i] = acc;
  }
}

// adds the diagonal, then sum c*sigma and sum c^2 (exact) per state
__global__ __launch_bounds__(BLK) void k_energy_reduce(Compact cp, Counters* cnt, const double* __restrict__ h1,
                                                       const double* __restrict__ h2, int n) {
  const uint64_t H = cp.cs;
  __shared__ double d1[32], Jt[32 * 32], Kt[32 * 32];  // n <= 32 spatial orbitals
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int P = e / n, Q = e - P * n;
    Jt[e] = eri(h2, n, P, P, Q, Q);
    Kt[e] = eri(h2, n, P, Q, Q, P);
  }
  for (int P = threadIdx.x; P < n; P += blockDim.x) d1[P] = h1[P * n + P];
  __syncthreads();
  const int b = blockIdx.y;
  const int64_t N = static_cast<int64_t>(cnt[b].ncompact);
  Fx num = fx_zero(), den = fx_zero();
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const double c = cp.amp[b * H + i];
    const double sig = cp.sig[b * H + i] + h_diag(cp.key[b * H + i], d1, Jt, Kt, n) * c;
    cp.sig[b * H + i] = sig;
    num = fx_add(num, fx_from(c * sig));
    den = fx_add(den, fx_from(c * c));
  }
  Red r;
  r.f = num;
  for (int q = 0; q < 7; ++q) r.c[q] = 0;
  r = block_reduce(r);
  ESum& es = cnt[b].es[blockIdx.x & (ESH - 1)];
  if (threadIdx.x == 0 && fx_nonzero(r.f)) fx3_atomic_add(&es.num, r.f);
  __syncthreads();
  r.f = den;
  r = block_reduce(r);
  if (threadIdx.x == 0 && fx_nonzero(r.f)) fx3_atomic_add(&es.den, r.f);
}



// ---------------------------------------------------------------------------
// index growth: a larger index, rebuilt from the entries (which do not move)
// ---------------------------------------------------------------------------
__global__ void k_idx_clear(Tab t, Pf pf) {
  Idx* ix = t.idx + blockIdx.y * t.Hcap;
  for (uint64_t s = blockIdx.x * blockDim.x + threadIdx.x; s < t.H; s += gridDim.x * blockDim.x) {
    ix[s].key = EMPTY_KEY;
    ix[s].id = NO_ID;
    if (pf.w && s < pf.n) pf.w[blockIdx.y * pf.stride + s] = 0ull;
  }
}

// Every entry, alive or dead, is indexed (keys are unique, so every insert
// claims its own slot); the growth check stopped no step any more.
template <class T>
__global__ void k_reindex(Tab t, Counters* cnt, Pf pf) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int a = scan_arena();
  const uint64_t n = t.ac[b * NA + a];
  for (uint64_t j = scan_rank() * BLK + threadIdx.x; j < n; j += scan_blocks() * BLK) {
    const uint64_t key = v.sl[a * v.A + j].key;
    if (!index_insert(v.ix, v.H, key, home_slot(key, v.H), entry_id(a, j)))
      atomicOr(&cnt[b].flags, F_TABLE_FULL);
    else
      pf_add(pf, b, key);
  }
  if (b == 0 && blockIdx.x == 0 && threadIdx.x == 0) cnt[0].stop = ~0u;
}

// Entry positions the last sweeps scanned (statistics): the forward
// launches' counts at their start (every arena of a launch is written
// together), and what undoing each factor scans; into C_FSCAN / C_RSCAN of
// shard 0.
__global__ void k_scan_totals(StepArr sa, Counters* cnt, int64_t M) {
  const int b = blockIdx.x;
  unsigned long long f = 0, r = 0;
  for (int64_t k = 1 + threadIdx.x; k <= M; k += blockDim.x) {
    const int64_t row = (static_cast<int64_t>(b) * sa.nstride + k) * NA;
    if (sa.nb[row] != NB_UNSET)
      for (int a = 0; a < NA; ++a) f += sa.nb[row + a];
    for (int a = 0; a < NA; ++a) {
      const uint32_t n1 = sa.nb[row + NA + a];
      r += n1 != NB_UNSET ? n1 : sa.nb[row + 2 * NA + a];
    }
  }
  __shared__ unsigned long long part[2][BLK / 64];
  f = wave_u64(f);
  r = wave_u64(r);
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = f;
    part[1][threadIdx.x >> 6] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tf = 0, tr = 0;
    for (int w = 0; w < BLK / 64; ++w) {
      tf += part[0][w];
      tr += part[1][w];
    }
    cnt[b].sh[0].v[C_FSCAN] = tf;
    cnt[b].sh[0].v[C_RSCAN] = tr;
  }
}

// Counters of a fresh state: everything zero, the scale S0, no stop step.
// One block per batch member, each lane writing whole 8-byte words.
static_assert(sizeof(Counters) % 8 == 0 && offsetof(Counters, S) % 8 == 0, "Counters word layout");
static_assert(offsetof(Counters, flags) % 8 == 0 && offsetof(Counters, stop) == offsetof(Counters, flags) + 4,
              "flags and stop share one word");
__global__ void k_counters_reset(Counters* cnt, double S0) {
  unsigned long long* w = reinterpret_cast<unsigned long long*>(cnt + blockIdx.x);
  constexpr unsigned int nw = sizeof(Counters) / 8;
  constexpr unsigned int w_stop = offsetof(Counters, flags) / 8, w_s = offsetof(Counters, S) / 8;
  for (unsigned int i = threadIdx.x; i < nw; i += blockDim.x)
    w[i] = i == w_stop ? (0xffffffffull << 32) : i == w_s ? static_cast<unsigned long long>(__double_as_longlong(S0))
                                                            : 0ull;
}

// The live and entry counts of a state about to be refilled.
__global__ void k_counters_live_reset(Counters* cnt) {
  if (threadIdx.x < CSH) {
    cnt[blockIdx.x].sh[threadIdx.x].v[C_LIVE] = 0ull;
    cnt[blockIdx.x].sh[threadIdx.x].v[C_OCC] = 0ull;
  }
}

__global__ void k_energy_begin(Counters* cnt, int B) {
  const int b = threadIdx.x;
  if (b >= B) return;
  cnt[b].ncompact = 0;
  cnt[b].num = fx_zero();
  cnt[b].den = fx_zero();
  for (int q = 0; q < ESH; ++q) {
    cnt[b].es[q].num = fx3_zero();
    cnt[b].es[q].den = fx3_zero();
  }
}

__global__ void k_energy_final(Counters* cnt, double* E, int B) {
  const int b = threadIdx.x;
  if (b >= B) return;
  Fx num = fx_zero(), den = fx_zero();
  for (int q = 0; q < ESH; ++q) {
    num = fx_add(num, fx3_value(cnt[b].es[q].num));
    den = fx_add(den, fx3_value(cnt[b].es[q].den));
  }
  cnt[b].num = num;
  cnt[b].den = den;
  const double e = fx_to_d(num) / fx_to_d(den);
  cnt[b].E = e;
  if (E) E[b] = e;
}

// lambda_M = P_M (H - E) psi_M on the support (raw amplitudes)
template <class T>
__global__ void k_lambda(Tab t, Compact cp, const Counters* cnt) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int64_t N = static_cast<int64_t>(cnt[b].ncompact);
  const double E = cnt[b].E;
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const double x = cp.sig[b * cp.cs + i] - E * cp.amp[b * cp.cs + i];
    v.lam(v.off(cp.slot[b * cp.cs + i])) = static_cast<T>(x);
  }
}

// dE/dtheta_k = 2 <w|A_k psi> / <psi|psi>: one wave per step, lane q adding
// shard q (exact sums, so the grouping changes nothing)
static_assert(SH == 64, "one lane per gradient shard");
__global__ void k_grad_final(StepArr sa, const Counters* cnt, double* grad, int64_t M) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * (BLK / 64) + (threadIdx.x >> 6);  // uniform in a wave
  const Fx v = k < M ? fx3_value(sa.gacc[sidx(sa, b, lane, k + 1)]) : fx_zero();
  const Fx g = wave_fx(v);
  if (lane == 0 && k < M) grad[b * M + k] = 2.0 * fx_to_d(g) / fx_to_d(cnt[b].den);
}


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int grid_for(uint64_t work, int block, int cap) {
  uint64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > static_cast<uint64_t>(cap)) g = cap;
  return static_cast<int>(g);
}

void launch_fill(const Tab& t, int B, hipStream_t st, const Pf& pf) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(t.H, BLK, 8192), B), dim3(BLK), 0, st, t, pf);
}

// Checks a list that k_insert_list put into member 0: every key a
// determinant of nq qubits, every amplitude finite, and every key indexed
// under its own entry (a key given twice is found under one of its entries
// only, so the other fails the check).
__global__ void k_check_list(Tab t, Counters* cnt, const uint64_t* __restrict__ keys,
                             const double* __restrict__ amps, int64_t n, int nq) {
  const uint64_t high = nq >= 64 ? 0ull : (~0ull << nq);
  bool bad = false;
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint64_t key = keys[i];
    if (key == EMPTY_KEY || (key & high) || !isfinite(amps[i])) {
      bad = true;
      continue;
    }
    uint64_t ff;
    Idx iv;
    if (find_slot(t.idx, t.H, key, &ff, &iv) < 0 || iv.id != entry_id(static_cast<int>(i % NA), i / NA)) bad = true;
  }
  if (bad) atomicOr(&cnt[0].flags, F_BAD_INPUT);
}

void launch_check_list(const Tab& t, Counters* cnt, const uint64_t* keys, const double* amps, int64_t n, int nq,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_check_list, dim3(grid_for(n > 0 ? n : 1, BLK, 4096)), dim3(BLK), 0, st, t, cnt, keys, amps,
                     n, nq);
}

template <class T>
void launch_insert_list(const Tab& t, Counters* cnt, const uint64_t* keys, const double* amps, int64_t n_fixed,
                        uint64_t stride, int64_t nmax, int B, hipStream_t st, const Pf& pf) {
  hipLaunchKernelGGL(k_insert_list<T>, dim3(grid_for(nmax > 0 ? nmax : 1, BLK, 4096), B), dim3(BLK), 0, st, t, cnt,
                     keys, amps, n_fixed, stride, pf);
}

void launch_trig(const double* theta, Trig* trig, int64_t M, int64_t ld, int B, Counters* cnt, hipStream_t st) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_trig, dim3(grid_for(M, BLK, 1024), B), dim3(BLK), 0, st, theta, trig, M, ld, cnt);
}

template <class T>
void launch_sweep_begin(const Tab& t, const StepArr& sa, Counters* cnt, int64_t M, int B, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_sweep_begin<T>, dim3(grid, B), dim3(BLK), 0, st, t, sa, cnt, M);
}

void launch_sweep_end(const Tab& t, const StepArr& sa, Counters* cnt, int64_t M, int64_t k_last, int B,
                      const Sync* sy, int fold_only, hipStream_t st) {
  hipLaunchKernelGGL(k_sweep_end, dim3(B), dim3(BLK), 0, st, t, sa, cnt, M, k_last, sy, fold_only);
}

void launch_sync_reset(Sync* sy, int clear_timeout, hipStream_t st) {
  hipLaunchKernelGGL(k_sync_reset, dim3(1), dim3(64), 0, st, sy, clear_timeout);
}

template <class T>
int resident_blocks_per_cu(int which) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (which) {
    case 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_sweep<T>, BLK, 0); break;
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rev_sweep<T>, BLK, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd<T, false>, BLK, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rev<T>, BLK, 0); break;
    case 5: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd2<T, PH2>, BLK, 0); break;
    case 6: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rev2<T, PH2>, BLK, 0); break;
    case 7: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fwd_ho<T>, BLK, 0); break;
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

template <class T>
hipError_t launch_fwd_sweep(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa,
                            Counters* cnt, const LogArr& lg, int k0, int k1, double thr, int prune_first, int log_on,
                            Sync* sy, int B, int grid, hipStream_t st) {
  Tab a_t = t;
  const FacMask* a_fac = fac;
  const Trig* a_trig = trig;
  int64_t a_ld = ld;
  StepArr a_sa = sa;
  Counters* a_cnt = cnt;
  LogArr a_lg = lg;
  int a_k0 = k0, a_k1 = k1, a_pf = prune_first, a_log = log_on;
  double a_thr = thr;
  Sync* a_sy = sy;
  void* args[] = {&a_t, &a_fac, &a_trig, &a_ld, &a_sa, &a_cnt, &a_lg, &a_k0, &a_k1, &a_thr, &a_pf, &a_log, &a_sy};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_fwd_sweep<T>), dim3(grid, B), dim3(BLK), args,
                                    0, st);
}

template <class T>
hipError_t launch_rev_sweep(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa,
                            Counters* cnt, const LogArr& lg, int k_hi, int k_lo, Sync* sy, int B, int grid,
                            hipStream_t st) {
  Tab a_t = t;
  const FacMask* a_fac = fac;
  const Trig* a_trig = trig;
  int64_t a_ld = ld;
  StepArr a_sa = sa;
  Counters* a_cnt = cnt;
  LogArr a_lg = lg;
  int a_hi = k_hi, a_lo = k_lo;
  Sync* a_sy = sy;
  void* args[] = {&a_t, &a_fac, &a_trig, &a_ld, &a_sa, &a_cnt, &a_lg, &a_hi, &a_lo, &a_sy};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_rev_sweep<T>), dim3(grid, B), dim3(BLK), args,
                                    0, st);
}

template <class T>
void launch_fwd(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                const LogArr& lg, int k, double thr, int prune_all, int log_on, uint64_t occ_lim, int B, int grid,
                int split, int hiocc, const Pf& pf, hipStream_t st) {
  const int nl = split ? B : 1, gy = split ? 1 : B;
  for (int b0 = 0; b0 < nl; ++b0) {
    if (sa.ea)
      hipLaunchKernelGGL((k_fwd<T, true>), dim3(grid, gy), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, lg, k, thr,
                         prune_all, log_on, occ_lim, b0, B);
    else if (hiocc && pf.w)
      hipLaunchKernelGGL(k_fwd_ho_pf<T>, dim3(grid, gy), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, lg, k, thr,
                         prune_all, log_on, occ_lim, b0, B, pf);
    else if (hiocc)
      hipLaunchKernelGGL(k_fwd_ho<T>, dim3(grid, gy), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, lg, k, thr,
                         prune_all, log_on, occ_lim, b0, B);
    else if (pf.w)
      hipLaunchKernelGGL(k_fwd_pf<T>, dim3(grid, gy), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, lg, k, thr,
                         prune_all, log_on, occ_lim, b0, B, pf);
    else
      hipLaunchKernelGGL((k_fwd<T, false>), dim3(grid, gy), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, lg, k, thr,
                         prune_all, log_on, occ_lim, b0, B);
  }
}

template <class T>
void launch_rev(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                int k, int B, int grid, int split, const Pf& pf, hipStream_t st) {
  const int nl = split ? B : 1, gy = split ? 1 : B;
  for (int b0 = 0; b0 < nl; ++b0) {
    if (pf.w)
      hipLaunchKernelGGL(k_rev_pf<T>, dim3(grid, gy), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, k, b0, pf);
    else
      hipLaunchKernelGGL(k_rev<T>, dim3(grid, gy), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, k, b0);
  }
}

template <class T>
void launch_fwd2(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                 int k, int B, int grid, int wide, hipStream_t st) {
  // wide: PH2 index slots from every home loaded up front (the caller chooses
  // it when the launch covers the state in one pass with all its blocks
  // resident); otherwise the home slot only, keeping more waves resident
  if (wide)
    hipLaunchKernelGGL((k_fwd2<T, PH2>), dim3(grid, B), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, k);
  else
    hipLaunchKernelGGL((k_fwd2<T, 1>), dim3(grid, B), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, k);
}

template <class T>
void launch_rev2(const Tab& t, const FacMask* fac, const Trig* trig, int64_t ld, const StepArr& sa, Counters* cnt,
                 int k, int B, int grid, int wide, hipStream_t st) {
  if (wide)
    hipLaunchKernelGGL((k_rev2<T, PH2>), dim3(grid, B), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, k);
  else
    hipLaunchKernelGGL((k_rev2<T, 1>), dim3(grid, B), dim3(BLK), 0, st, t, fac, trig, ld, sa, cnt, k);
}

template <class T>
void launch_log_restore(const Tab& t, const LogArr& lg, const StepArr& sa, int k, int B, uint32_t maxcnt,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_log_restore<T>, dim3(grid_for(maxcnt, BLK, 1024), B), dim3(BLK), 0, st, t, lg, sa, k);
}

template <class T>
void launch_compact(const Tab& t, const Compact& cp, Counters* cnt, int B, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_compact<T>, dim3(grid, B), dim3(BLK), 0, st, t, cp, cnt);
}

template <class T>
void launch_snapshot(const Tab& t, const StepArr& sa, const Snap& sn, int k, int B, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_snapshot<T>, dim3(grid, B), dim3(BLK), 0, st, t, sa, sn, k);
}

template <class T>
void launch_snap_restore(const Tab& t, const Snap& sn, Counters* cnt, uint64_t nmax, int B, hipStream_t st) {
  if (nmax == 0) return;
  hipLaunchKernelGGL(k_snap_restore<T>, dim3(grid_for(nmax, BLK, 4096), B), dim3(BLK), 0, st, t, sn, cnt);
}

template <class T>
void launch_entropy_scan(const Tab& t, const StepArr& sa, int k, int B, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_entropy_scan<T>, dim3(grid, B), dim3(BLK), 0, st, t, sa, k);
}

void launch_entropy_final(const StepArr& sa, int64_t M, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_entropy_final, dim3(grid_for(static_cast<uint64_t>(M + 1), BLK, 1024), B), dim3(BLK), 0, st,
                     sa, M);
}

template <class T>
void launch_topk(const Tab& t, const StepArr& sa, Counters* cnt, TopK* tk, int k, uint64_t n_max, uint64_t n_cut,
                 int B, int grid, hipStream_t st) {
  constexpr int npass = (rank_bits<T>() + TK_BITS - 1) / TK_BITS;
  const unsigned long long nm = n_max, nc = n_cut;
  for (int pass = 0; pass < npass; ++pass)
    hipLaunchKernelGGL(k_topk_pass<T>, dim3(grid, B), dim3(BLK), 0, st, t, sa, tk, cnt, k, pass, nm, nc);
  hipLaunchKernelGGL(k_topk_kill<T>, dim3(grid, B), dim3(BLK), 0, st, t, sa, cnt, tk, k, nm, nc);
}

void launch_zero_u64(unsigned long long* p, uint64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n, BLK, 256)), dim3(BLK), 0, st, p, n);
}

template <class T>
void launch_sigma(const Tab& t, const Compact& cp, const Counters* cnt, const double* h1, const double* h2, int nq,
                  int64_t nmax, int B, int singles_only, hipStream_t st) {
  if (nmax <= 0) return;
  hipLaunchKernelGGL(k_sigma<T>, dim3(grid_for(static_cast<uint64_t>(nmax) * SG, BLK, 16384), B), dim3(BLK), 0, st,
                     t, cp, cnt, h1, h2, nq, singles_only);
}

void launch_energy_reduce(const Compact& cp, Counters* cnt, const double* h1, const double* h2, int n, int64_t nmax,
                          int B, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_reduce, dim3(grid_for(nmax, BLK, 2048), B), dim3(BLK), 0, st, cp, cnt, h1, h2, n);
}

void launch_counters_reset(Counters* cnt, int B, double S0, hipStream_t st) {
  hipLaunchKernelGGL(k_counters_reset, dim3(B), dim3(BLK), 0, st, cnt, S0);
}

void launch_scan_totals(const StepArr& sa, Counters* cnt, int64_t M, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_totals, dim3(B), dim3(BLK), 0, st, sa, cnt, M);
}

void launch_counters_live_reset(Counters* cnt, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_counters_live_reset, dim3(B), dim3(64), 0, st, cnt);
}

void launch_energy_begin(Counters* cnt, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_begin, dim3(1), dim3(64 * ((B + 63) / 64)), 0, st, cnt, B);
}

template <class T>
void launch_reindex(const Tab& t, Counters* cnt, int B, int grid, hipStream_t st, const Pf& pf) {
  hipLaunchKernelGGL(k_idx_clear, dim3(grid_for(t.H, BLK, 8192), B), dim3(BLK), 0, st, t, pf);
  hipLaunchKernelGGL(k_reindex<T>, dim3(grid, B), dim3(BLK), 0, st, t, cnt, pf);
}

// The filter rebuilt from every entry of every member (after steps that did
// not keep it): cleared, then every key's bits set.
__global__ void k_pf_clear(Pf pf) {
  for (uint64_t s = blockIdx.x * blockDim.x + threadIdx.x; s < pf.n; s += gridDim.x * blockDim.x)
    pf.w[blockIdx.y * pf.stride + s] = 0ull;
}

template <class T>
__global__ void k_pf_fill(Tab t, Pf pf) {
  const int b = blockIdx.y;
  const View<T> v = view<T>(t, b);
  const int a = scan_arena();
  const uint64_t n = t.ac[b * NA + a];
  for (uint64_t j = scan_rank() * BLK + threadIdx.x; j < n; j += scan_blocks() * BLK) pf_add(pf, b, v.sl[a * v.A + j].key);
}

template <class T>
void launch_pf_build(const Tab& t, const Pf& pf, int B, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_pf_clear, dim3(grid_for(pf.n, BLK, 8192), B), dim3(BLK), 0, st, pf);
  hipLaunchKernelGGL(k_pf_fill<T>, dim3(grid, B), dim3(BLK), 0, st, t, pf);
}

void launch_energy_final(Counters* cnt, double* E, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64 * ((B + 63) / 64)), 0, st, cnt, E, B);
}

template <class T>
void launch_lambda(const Tab& t, const Compact& cp, const Counters* cnt, int64_t nmax, int B, hipStream_t st) {
  hipLaunchKernelGGL(k_lambda<T>, dim3(grid_for(nmax, BLK, 4096), B), dim3(BLK), 0, st, t, cp, cnt);
}

void launch_grad_final(const StepArr& sa, const Counters* cnt, double* grad, int64_t M, int B, hipStream_t st) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_grad_final, dim3(static_cast<unsigned int>((M + BLK / 64 - 1) / (BLK / 64)), B), dim3(BLK), 0, st,
                     sa, cnt, grad, M);
}

// ---------------------------------------------------------------------------
// sigma, double excitations, by pairing (a sort instead of hash probes)
// ---------------------------------------------------------------------------
// I and J differ by a double excitation exactly when removing two occupied
// spin-orbitals from each leaves the same (N-2)-electron pattern K, the
// removed pairs being disjoint.  Every determinant emits one record (K, i) per
// pair of its occupied spin-orbitals; records sorted by K form groups, and a
// record's share of sigma_I is the sum over the other members J of its group
// with a disjoint removed pair of <I|H|J> c_J.  Each double connection present
// in the state is met exactly once from each side, and nothing absent is
// probed.  Partial sums are exact fixed point, so the order of a group does
// not matter; records are split into partitions by a hash of K to bound the
// scratch memory.

constexpr int RS_ITEMS = 16;             // elements per thread of a sort tile
constexpr int RS_TILE = BLK * RS_ITEMS;  // elements per block of a sort pass
constexpr int SCAN_CH = BLK * 16;        // scan chunk

__device__ __forceinline__ int pair_part(uint64_t K, int nparts) {
  return static_cast<int>((mix64(K) >> 40) % static_cast<uint64_t>(nparts));
}

// digit histogram of every tile: hist[digit * blocks + block]
__global__ __launch_bounds__(BLK) void k_rs_hist(const uint64_t* __restrict__ keys, uint64_t n, int shift,
                                                 uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint64_t e = base + static_cast<uint64_t>(r) * BLK + threadIdx.x;
    if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[static_cast<uint64_t>(threadIdx.x) * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of 256 values held one per thread (block-wide)
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  tmp[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < BLK; o <<= 1) {
    const uint32_t add = threadIdx.x >= static_cast<unsigned>(o) ? tmp[threadIdx.x - o] : 0u;
    __syncthreads();
    tmp[threadIdx.x] += add;
    __syncthreads();
  }
  const uint32_t incl = tmp[threadIdx.x];
  *total = tmp[BLK - 1];
  __syncthreads();
  return incl - v;
}

// exclusive scan of each SCAN_CH chunk in place; chunk totals into sums
__global__ __launch_bounds__(BLK) void k_scan_local(uint32_t* __restrict__ a, uint64_t L, uint32_t* __restrict__ sums) {
  __shared__ uint32_t tmp[BLK];
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * SCAN_CH + static_cast<uint64_t>(threadIdx.x) * 16;
  uint32_t v[16], tsum = 0;
  for (int j = 0; j < 16; ++j) {
    v[j] = base + j < L ? a[base + j] : 0u;
    tsum += v[j];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(tsum, tmp, &total);
  for (int j = 0; j < 16; ++j) {
    if (base + j < L) a[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of the chunk totals (one block, nchunks <= BLK * 16)
__global__ __launch_bounds__(BLK) void k_scan_top(uint32_t* __restrict__ sums, uint64_t nchunks) {
  __shared__ uint32_t tmp[BLK];
  const uint64_t base = static_cast<uint64_t>(threadIdx.x) * 16;
  uint32_t v[16], tsum = 0;
  for (int j = 0; j < 16; ++j) {
    v[j] = base + j < nchunks ? sums[base + j] : 0u;
    tsum += v[j];
  }
  uint32_t total;
  uint32_t run = block_exclusive_scan(tsum, tmp, &total);
  for (int j = 0; j < 16; ++j) {
    if (base + j < nchunks) sums[base + j] = run;
    run += v[j];
  }
}

__global__ void k_scan_add(uint32_t* __restrict__ a, uint64_t L, const uint32_t* __restrict__ sums) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < L;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    a[i] += sums[i / SCAN_CH];
}

// stable scatter of one radix pass: a tile is taken RS_ITEMS times 256
// elements in order; lanes with equal digits are ranked by ballots, waves by
// LDS counts
__global__ __launch_bounds__(BLK) void k_rs_scatter(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                    uint64_t n, int shift, const uint32_t* __restrict__ offs) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[BLK / 64][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = offs[static_cast<uint64_t>(t) * gridDim.x + blockIdx.x];
  for (int q = 0; q < BLK / 64; ++q) wcnt[q][t] = 0u;
  __syncthreads();
  const uint64_t base = static_cast<uint64_t>(blockIdx.x) * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const uint64_t e = base + static_cast<uint64_t>(r) * BLK + t;
    const bool valid = e < n;
    const uint64_t key = valid ? kin[e] : 0ull;
    const uint32_t val = valid ? vin[e] : 0u;
    const uint32_t d = static_cast<uint32_t>(key >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (d >> bit) & 1u;
      const unsigned long long bb = __ballot(on);
      peers &= on ? bb : ~bb;
    }
    const uint32_t rank = static_cast<uint32_t>(__popcll(peers & ((1ull << lane) - 1ull)));
    if (valid && rank == 0) wcnt[w][d] = static_cast<uint32_t>(__popcll(peers));
    __syncthreads();
    if (valid) {
      uint32_t pre = 0;
      for (int q = 0; q < w; ++q) pre += wcnt[q][d];
      const uint32_t pos = run[d] + pre + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < BLK / 64; ++q) {
      add += wcnt[q][t];
      wcnt[q][t] = 0u;
    }
    run[t] += add;
    __syncthreads();
  }
}

// records (K, i) of partition `part` for determinants i < N of member b
// Records (K, i) of determinant i for every K = I with `order` (1 or 2)
// electrons removed, in the hash partition `part`.
__global__ __launch_bounds__(BLK) void k_pair_emit(Compact cp, uint64_t H, int b, uint64_t N, int part, int nparts,
                                                   uint64_t* __restrict__ rk, uint32_t* __restrict__ ri,
                                                   unsigned long long* __restrict__ count, uint64_t cap, int order) {
  const int lane = threadIdx.x & 63;
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  // loop bound uniform across the wave so the ballot-free prefix below is safe
  for (uint64_t i0 = blockIdx.x * static_cast<uint64_t>(blockDim.x) + (threadIdx.x & ~63u); i0 < N; i0 += stride) {
    const uint64_t i = i0 + lane;
    const uint64_t I = i < N ? cp.key[b * H + i] : 0ull;
    unsigned int c = 0;
    for (uint64_t m1 = I; m1; m1 &= m1 - 1ull) {
      const uint64_t b1 = m1 & (~m1 + 1ull);
      if (order == 1) {
        c += pair_part(I ^ b1, nparts) == part;
        continue;
      }
      for (uint64_t m2 = m1 & (m1 - 1ull); m2; m2 &= m2 - 1ull)
        c += pair_part(I ^ b1 ^ (m2 & (~m2 + 1ull)), nparts) == part;
    }
    // wave prefix of the counts, one atomic per wave
    unsigned int incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const unsigned int tot = __shfl(incl, 63, 64);
    unsigned long long basep = 0;
    if (lane == 63 && tot) basep = atomicAdd(count, static_cast<unsigned long long>(tot));
    basep = __shfl(basep, 63, 64);
    uint64_t pos = basep + incl - c;
    for (uint64_t m1 = I; m1; m1 &= m1 - 1ull) {
      const uint64_t b1 = m1 & (~m1 + 1ull);
      if (order == 1) {
        const uint64_t K = I ^ b1;
        if (pair_part(K, nparts) != part) continue;
        if (pos < cap) {
          rk[pos] = K;
          ri[pos] = static_cast<uint32_t>(i);
        }
        ++pos;
        continue;
      }
      for (uint64_t m2 = m1 & (m1 - 1ull); m2; m2 &= m2 - 1ull) {
        const uint64_t K = I ^ b1 ^ (m2 & (~m2 + 1ull));
        if (pair_part(K, nparts) != part) continue;
        if (pos < cap) {
          rk[pos] = K;
          ri[pos] = static_cast<uint32_t>(i);
        }
        ++pos;
      }
    }
  }
}

// each sorted record: its determinant and amplitude, next to it
__global__ void k_pair_gather(Compact cp, uint64_t H, int b, const uint32_t* __restrict__ ri, uint64_t n,
                              uint64_t* __restrict__ rI, double* __restrict__ rc) {
  for (uint64_t j = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; j < n;
       j += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    rI[j] = cp.key[b * H + ri[j]];
    rc[j] = cp.amp[b * H + ri[j]];
  }
}

// a record's share of sigma: the other members of its group (same K) whose
// removed electrons are disjoint from its own (order 2: the doubles; order 1:
// every other member, a single excitation).  A wave takes 64 consecutive
// records: group bounds come from wave scans of the group heads and tails,
// with a walk only for the groups that cross the wave's edges; members are
// read four at a time so their loads are in flight together.
__global__ __launch_bounds__(BLK) void k_pair_sigma(const uint64_t* __restrict__ K, const uint64_t* __restrict__ rI,
                                                    const double* __restrict__ rc, const uint32_t* __restrict__ ri,
                                                    uint64_t n, const double* __restrict__ h1,
                                                    const double* __restrict__ h2, int n_orb,
                                                    Fx3* __restrict__ acc, int order) {
  const int lane = threadIdx.x & 63;
  const uint64_t wstride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t j0 = blockIdx.x * static_cast<uint64_t>(blockDim.x) + (threadIdx.x & ~63u); j0 < n; j0 += wstride) {
    const uint64_t j = j0 + lane;
    const bool valid = j < n;
    const uint64_t k = valid ? K[j] : ~0ull;
    const bool head = valid && (j == 0 || K[j - 1] != k);
    const bool tail = valid && (j + 1 == n || K[j + 1] != k);
    // start: last head at or before this lane; end: first tail at or after it
    long long sv = head ? static_cast<long long>(j) : -1;
    unsigned long long ev = tail ? j + 1 : ~0ull;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const long long a = __shfl_up(sv, o, 64);
      if (lane >= o && a > sv) sv = a;
      const unsigned long long c = __shfl_down(ev, o, 64);
      if (lane + o < 64 && c < ev) ev = c;
    }
    if (!valid) continue;
    uint64_t s0 = sv >= 0 ? static_cast<uint64_t>(sv) : j0;
    if (sv < 0) while (s0 > 0 && K[s0 - 1] == k) --s0;  // group began in an earlier wave
    uint64_t e0 = ev != ~0ull ? ev : j0 + 64;
    if (ev == ~0ull) while (e0 < n && K[e0] == k) ++e0;  // group goes on past this wave
    if (e0 - s0 < 2) continue;
    const uint64_t I = rI[j], dI = I ^ k;
    Fx a = fx_zero();
    for (uint64_t u0 = s0; u0 < e0; u0 += 4) {
      uint64_t J[4];
      double c[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint64_t u = u0 + q;
        J[q] = u < e0 ? rI[u] : I;
        c[q] = u < e0 ? rc[u] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // same determinant, or (order 2) a shared removed orbital: a single,
        // which the one-electron groups count
        if (J[q] == I || ((J[q] ^ k) & dI)) continue;
        a = fx_add(a, fx_from(h_offdiag(I, J[q], 2 * order, h1, h2, n_orb) * c[q]));
      }
    }
    if (fx_nonzero(a)) fx3_atomic_add(&acc[ri[j]], a);
  }
}

// sigma of the off-diagonal part, summed exactly over both kinds of groups
__global__ void k_pair_finish(Compact cp, uint64_t H, int b, uint64_t N, Fx3* __restrict__ acc) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < N;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    cp.sig[b * H + i] = fx_to_d(fx3_value(acc[i]));
    acc[i] = fx3_zero();
  }
}

void launch_pair_emit(const Compact& cp, uint64_t H, int b, uint64_t N, int part, int nparts, uint64_t* rk,
                      uint32_t* ri, unsigned long long* count, uint64_t cap, int order, hipStream_t st) {
  hipLaunchKernelGGL(k_pair_emit, dim3(grid_for(N, BLK, 8192)), dim3(BLK), 0, st, cp, H, b, N, part, nparts, rk, ri,
                     count, cap, order);
}

// LSD radix sort of (key, value) by the low `bits` bits of the key, 8 per
// pass, ping-ponging between (k0, v0) and (k1, v1); returns 1 when the
// result ended in (k1, v1)
int launch_radix_sort(uint64_t* k0, uint32_t* v0, uint64_t* k1, uint32_t* v1, uint64_t n, int bits, uint32_t* hist,
                      uint32_t* sums, hipStream_t st) {
  if (n == 0) return 0;
  const uint64_t nblk = (n + RS_TILE - 1) / RS_TILE;
  const uint64_t L = 256 * nblk;
  const uint64_t nch = (L + SCAN_CH - 1) / SCAN_CH;
  int flip = 0;
  for (int shift = 0; shift < bits; shift += 8) {
    uint64_t* ki = flip ? k1 : k0;
    uint32_t* vi = flip ? v1 : v0;
    uint64_t* ko = flip ? k0 : k1;
    uint32_t* vo = flip ? v0 : v1;
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(BLK), 0, st, ki, n, shift, hist);
    hipLaunchKernelGGL(k_scan_local, dim3(nch), dim3(BLK), 0, st, hist, L, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(BLK), 0, st, sums, nch);
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(L, BLK, 4096)), dim3(BLK), 0, st, hist, L, sums);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(BLK), 0, st, ki, vi, ko, vo, n, shift, hist);
    flip ^= 1;
  }
  return flip;
}

void launch_pair_groups(const Compact& cp, uint64_t H, int b, const uint64_t* K, const uint32_t* ri, uint64_t n,
                        uint64_t* rI, double* rc, const double* h1, const double* h2, int n_orb, Fx3* acc,
                        int order, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_pair_gather, dim3(grid_for(n, BLK, 8192)), dim3(BLK), 0, st, cp, H, b, ri, n, rI, rc);
  hipLaunchKernelGGL(k_pair_sigma, dim3(grid_for(n, BLK, 16384)), dim3(BLK), 0, st, K, rI, rc, ri, n, h1, h2, n_orb,
                     acc, order);
}

void launch_pair_finish(const Compact& cp, uint64_t H, int b, uint64_t N, Fx3* acc, hipStream_t st) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_pair_finish, dim3(grid_for(N, BLK, 4096)), dim3(BLK), 0, st, cp, H, b, N, acc);
}

void launch_fx3_zero(Fx3* a, uint64_t n, hipStream_t st) {
  if (n == 0) return;
  launch_zero_u64(reinterpret_cast<unsigned long long*>(a), 3 * n, st);
}

#define SWC_INST(T)                                                                                                \
  template void launch_insert_list<T>(const Tab&, Counters*, const uint64_t*, const double*, int64_t, uint64_t,   \
                                      int64_t, int, hipStream_t, const Pf&);                                       \
  template void launch_sweep_begin<T>(const Tab&, const StepArr&, Counters*, int64_t, int, int, hipStream_t);     \
  template void launch_fwd<T>(const Tab&, const FacMask*, const Trig*, int64_t, const StepArr&, Counters*,        \
                              const LogArr&, int, double, int, int, uint64_t, int, int, int, int, const Pf&,      \
                              hipStream_t);                                                                        \
  template void launch_rev<T>(const Tab&, const FacMask*, const Trig*, int64_t, const StepArr&, Counters*, int,   \
                              int, int, int, const Pf&, hipStream_t);                                              \
  template void launch_pf_build<T>(const Tab&, const Pf&, int, int, hipStream_t);                                 \
  template void launch_log_restore<T>(const Tab&, const LogArr&, const StepArr&, int, int, uint32_t,              \
                                      hipStream_t);                                                                \
  template void launch_compact<T>(const Tab&, const Compact&, Counters*, int, int, hipStream_t);                  \
  template void launch_lambda<T>(const Tab&, const Compact&, const Counters*, int64_t, int, hipStream_t);        \
  template void launch_sigma<T>(const Tab&, const Compact&, const Counters*, const double*, const double*, int,   \
                                int64_t, int, int, hipStream_t);                                                   \
  template int resident_blocks_per_cu<T>(int);                                                                    \
  template hipError_t launch_fwd_sweep<T>(const Tab&, const FacMask*, const Trig*, int64_t, const StepArr&,       \
                                          Counters*, const LogArr&, int, int, double, int, int, Sync*, int, int,   \
                                          hipStream_t);                                                            \
  template hipError_t launch_rev_sweep<T>(const Tab&, const FacMask*, const Trig*, int64_t, const StepArr&,       \
                                          Counters*, const LogArr&, int, int, Sync*, int, int, hipStream_t);      \
  template void launch_reindex<T>(const Tab&, Counters*, int, int, hipStream_t, const Pf&);                      \
  template void launch_fwd2<T>(const Tab&, const FacMask*, const Trig*, int64_t, const StepArr&, Counters*, int,  \
                               int, int, int, hipStream_t);                                                        \
  template void launch_rev2<T>(const Tab&, const FacMask*, const Trig*, int64_t, const StepArr&, Counters*, int,  \
                               int, int, int, hipStream_t);                                                        \
  template void launch_snapshot<T>(const Tab&, const StepArr&, const Snap&, int, int, int, hipStream_t);          \
  template void launch_entropy_scan<T>(const Tab&, const StepArr&, int, int, int, hipStream_t);                   \
  template void launch_topk<T>(const Tab&, const StepArr&, Counters*, TopK*, int, uint64_t, uint64_t, int, int,   \
                               hipStream_t);                                                                       \
  template void launch_snap_restore<T>(const Tab&, const Snap&, Counters*, uint64_t, int, hipStream_t);

SWC_INST(float)
SWC_INST(double)

}  // namespace swc
