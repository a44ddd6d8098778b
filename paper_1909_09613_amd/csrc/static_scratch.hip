// Allocation-free initialisation: a context whose scratch buffer (run tables,
// tile queue and segments, sort keys, diagnostic partial sums) is a
// file-scope device array instead of caller memory, for callers that cannot
// allocate device memory.  The caller still provides the particle, field and
// current buffers.
//
// The array is a host-side stand-in in host code: its device address is
// taken once per device with hipGetSymbolAddress, with that device current,
// and only that address is handed to the context.  One array per device, so
// at most one such context may be alive per device at a time; a second one
// is refused until the first is destroyed.
#include <cstdio>
#include <mutex>

#include "../../include/wtpic.h"
#include "launch.hpp"

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_addr[kMaxDevices];   // device address of the array on each device
bool g_busy[kMaxDevices];    // a context uses the device's array

void release_device(int dev) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (dev >= 0 && dev < kMaxDevices) g_busy[dev] = false;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

extern "C" pic_status pic_init_static(const pic_run_desc* runs, int32_t n_runs, const pic_buffers* bufs,
                                      void* hip_stream, pic_ctx** out) {
  if (!out || !bufs) {
    wtpic::set_global_error("out and bufs must not be NULL");
    return PIC_ERR_ARG;
  }
  size_t need[4] = {0, 0, 0, 0};
  pic_status st = pic_query_layout(runs, n_runs, need);
  if (st != PIC_OK) return st;
  if (need[3] > kStaticScratchBytes) {
    char msg[200];
    snprintf(msg, sizeof msg, "these runs need %zu bytes of scratch; the static scratch holds %zu", need[3],
             kStaticScratchBytes);
    wtpic::set_global_error(msg);
    return PIC_ERR_ARG;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    wtpic::set_global_error("hipGetDevice failed or device index too large");
    return PIC_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      wtpic::set_global_error("hipGetSymbolAddress of the static scratch failed");
      return PIC_ERR_HIP;
    }
    g_addr[dev] = p;
  }
  if (g_busy[dev]) {
    wtpic::set_global_error("another context of pic_init_static is alive on this device (one static scratch "
                            "per device)");
    return PIC_ERR_STATE;
  }
  pic_buffers b = *bufs;
  b.scratch = g_addr[dev];
  b.bytes[3] = kStaticScratchBytes;
  // pic_init clears every part of the scratch that must start at zero and
  // uploads the rest, so what an earlier context left there does not matter
  st = pic_init(runs, n_runs, &b, hip_stream, out);
  if (st == PIC_OK) {
    g_busy[dev] = true;
    wtpic::set_destroy_hook(*out, release_device, dev);
  }
  return st;
}
