// swc_energy_noalloc: the energy of a given state with no device allocation.
// Every scratch byte (index, entries, compact arrays, counters) lives in one
// file-scope device array, so the call suits callers that cannot allocate.
// The kernels are the ones swc_build_state + swc_energy run (FP64 amplitudes).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "swc.h"
#include "swc_internal.h"

namespace swc {
namespace {

constexpr int64_t NMAX = SWC_NOALLOC_MAX_DETS;
constexpr uint64_t HIDX = 4 * static_cast<uint64_t>(NMAX);  // index slots: at most 25% full
constexpr uint64_t AREN = static_cast<uint64_t>(NMAX) / NA;  // entries per arena (item i: arena i % NA)
static_assert(NMAX % NA == 0, "the determinants fill the arenas evenly");

constexpr size_t up256(size_t x) { return (x + 255) / 256 * 256; }
// layout of the scratch array: index | entries | compact key, amp, slot, sig | arena counts | counters
constexpr size_t OFF_IDX = 0;
constexpr size_t OFF_ENT = OFF_IDX + up256(sizeof(Idx) * HIDX);
constexpr size_t OFF_CKEY = OFF_ENT + up256(sizeof(Slot<double>) * NA * AREN);
constexpr size_t OFF_CAMP = OFF_CKEY + up256(8 * NMAX);
constexpr size_t OFF_CSLOT = OFF_CAMP + up256(8 * NMAX);
constexpr size_t OFF_CSIG = OFF_CSLOT + up256(4 * NMAX);
constexpr size_t OFF_AC = OFF_CSIG + up256(8 * NMAX);
constexpr size_t OFF_CNT = OFF_AC + up256(4 * NA);
constexpr size_t SCRATCH_BYTES = OFF_CNT + up256(sizeof(Counters));
static_assert(SCRATCH_BYTES == SWC_NOALLOC_SCRATCH_BYTES, "swc.h states the scratch size");

}  // namespace
}  // namespace swc

// The scratch of swc_energy_noalloc.  In host code this name is a host-side
// stand-in, not a device address: the kernels get the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[swc::SCRATCH_BYTES];

namespace swc {
namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};
int fail_na(int code, const char* msg) { return report_error(code, msg); }

// The device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int noalloc_scratch(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail_na(SWC_EDEVICE, "cannot query the current device");
  if (dev < 0 || dev >= MAX_DEVICES) return fail_na(SWC_EDEVICE, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail_na(SWC_EDEVICE, "hipGetSymbolAddress of the scratch array failed");
    g_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_ptr[dev]);
  return SWC_OK;
}

}  // namespace
}  // namespace swc

extern "C" int swc_energy_noalloc(int n_qubits, const uint64_t* dets, const double* amps, int64_t n,
                                  const double* h1, const double* h2, double* E, void* stream) {
  using namespace swc;
  if (n_qubits < 2 || n_qubits > 64 || (n_qubits & 1)) return fail_na(SWC_EINVAL, "n_qubits must be even, 2..64");
  if (n < 1) return fail_na(SWC_EINVAL, "empty state");
  if (n > NMAX) return fail_na(SWC_EINVAL, "state larger than the no-allocation scratch (65,536 determinants)");
  if (!dets || !amps || !h1 || !h2 || !E) return fail_na(SWC_EINVAL, "null pointer");
  char* w = nullptr;
  if (int r = noalloc_scratch(&w)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Tab t{w + OFF_ENT, nullptr, reinterpret_cast<Idx*>(w + OFF_IDX), reinterpret_cast<uint32_t*>(w + OFF_AC),
              HIDX, HIDX, AREN};
  const Compact cp{reinterpret_cast<uint64_t*>(w + OFF_CKEY), reinterpret_cast<double*>(w + OFF_CAMP),
                   reinterpret_cast<uint32_t*>(w + OFF_CSLOT), reinterpret_cast<double*>(w + OFF_CSIG),
                   static_cast<uint64_t>(NMAX)};
  Counters* cnt = reinterpret_cast<Counters*>(w + OFF_CNT);
  // The array keeps the last call's contents: everything read below is
  // written first (the index and arena counts by the fill, the counters by
  // their reset, the entries and compact arrays up to the counts).  Scale 1:
  // the energy is the Rayleigh quotient, whatever the norm.
  launch_fill(t, 1, st);
  launch_counters_reset(cnt, 1, 1.0, st);
  launch_insert_list<double>(t, cnt, dets, amps, n, 0, n, 1, st);
  launch_check_list(t, cnt, dets, amps, n, n_qubits, st);
  launch_energy_begin(cnt, 1, st);
  launch_compact<double>(t, cp, cnt, 1, NA, st);
  launch_sigma<double>(t, cp, cnt, h1, h2, n_qubits, n, 1, 0, st);
  launch_energy_reduce(cp, cnt, h1, h2, n_qubits / 2, n, 1, st);
  launch_energy_final(cnt, E, 1, st);
  if (hipGetLastError() != hipSuccess) return fail_na(SWC_EDEVICE, "kernel launch failed");
  // the status of the device-side checks (a small copy into host memory)
  Counters h{};
  if (hipMemcpyAsync(&h, cnt, sizeof(Counters), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail_na(SWC_EDEVICE, "device error");
  if (h.flags & F_BAD_INPUT)
    return fail_na(SWC_EINVAL, "a determinant is repeated or uses bits at or above n_qubits, or an amplitude is not finite");
  if (h.flags & F_TABLE_FULL) return fail_na(SWC_EDEVICE, "no-allocation index full");
  if (h.den.lo == 0 && h.den.hi == 0) return fail_na(SWC_EINVAL, "state has zero norm");
  return SWC_OK;
}
