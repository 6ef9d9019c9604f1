// Fixed device scratch for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): tsg_dense_eig_noalloc keeps the workspace of the batched small
// eigensolve in one file-scope device array instead of allocating it.
//
// Each GPU the library runs on holds its own copy of the array (64 MiB)
// until the process ends.  Host code never passes the array's name to a
// kernel: its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and that address is used.
// Every call on one GPU shares the array, so calls that overlap on one GPU
// (on different streams or threads) race.  Nothing in it has to start at
// zero: every region the eigensolve reads is written earlier in the same
// call (Z by the Householder accumulation, the reflector scalars by the
// Hessenberg reduction, the rotation log and its header by the chase).
#include <mutex>
#include <string>

#include "engine.h"

namespace tsg {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchElems = kScratchBytes / sizeof(c128);
static __device__ __align__(256) c128 scratch[kScratchElems];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
c128* g_addr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on first use).
c128* scratch_ptr() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) throw DeviceError("hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) throw DeviceError("device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw DeviceError(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_addr[dev] = static_cast<c128*>(p);
  }
  return g_addr[dev];
}

}  // namespace

int64_t noalloc_scratch_bytes() { return int64_t(kScratchBytes); }

void dense_eig_noalloc(void* H, int m, int batch, void* theta, void* Y, int* info, hipStream_t st) {
  if (!H || !theta || !Y || !info) throw InvalidArg("null device pointer");
  if (m < 1 || batch < 1) throw InvalidArg("need m >= 1 and batch >= 1");
  if (m > kMaxDenseBasis) throw InvalidArg("m exceeds the largest supported matrix (896)");
  const int64_t per = smalleig_workspace(m);
  if (per * batch > int64_t(kScratchElems))
    throw InvalidArg("batch x workspace(m) = " + std::to_string(per * batch * int64_t(sizeof(c128))) +
                     " bytes exceeds the fixed scratch of " + std::to_string(kScratchBytes) +
                     " bytes (use tsg_dense_eig, or fewer matrices per call)");
  c128* work = scratch_ptr();
  smalleig(static_cast<c128*>(H), int64_t(m) * m, m, static_cast<c128*>(theta), m, static_cast<c128*>(Y),
           int64_t(m) * m, work, per, info, batch, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw DeviceError(std::string("dense_eig_noalloc launch: ") + hipGetErrorString(e));
}

}  // namespace tsg
