// peps_qr_noalloc: the gauge QR of peps_qr with every piece of device
// workspace (kernel descriptors, the streaming kernel's workspace, the TSQR
// tree's row-block factors, split-K partial tiles of its rebuild) taken from
// one fixed device array per GPU instead of the memory pool, for callers
// that cannot allocate device memory.
#include <algorithm>
#include <mutex>

#include "../../include/peps_env.h"
#include "runtime.hpp"

namespace pe {
peps_status guarded_public(const std::function<void()>& f);

// The fixed workspace.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address (one per GPU) comes from
// hipGetSymbolAddress and only that address is ever passed on.
constexpr size_t NOALLOC_BYTES = size_t(PEPS_QR_NOALLOC_BYTES);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

}  // namespace

// Device address of this GPU's fixed workspace, looked up once per device
// with that device current (called when a context is created).
void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  PE_REQUIRE(device >= 0 && device < MAX_DEVICES, "device index beyond the fixed-workspace table");
  if (!g_scratch[device]) {
    int prev = 0;
    PE_HIP(hipGetDevice(&prev));
    PE_HIP(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    PE_HIP(hipSetDevice(prev));
    if (e != hipSuccess || p == nullptr)
      throw Error(ST_HIP, std::string("hipGetSymbolAddress of the fixed QR workspace failed: ") + hipGetErrorString(e));
    g_scratch[device] = p;
  }
  return g_scratch[device];
}

}  // namespace pe

using namespace pe;

extern "C" peps_status peps_qr_noalloc(peps_ctx* ctx, const peps_qr_block* blk, int32_t n_blocks) {
  return guarded_public([&] {
    PE_REQUIRE(ctx && blk, "ctx and blk must not be NULL");
    PE_REQUIRE(n_blocks >= 1, "n_blocks must be >= 1");
    for (int i = 0; i < n_blocks; ++i) {
      const peps_qr_block& b = blk[i];
      const std::string w = "block " + std::to_string(i) + ": ";
      PE_REQUIRE(b.a && b.q, w + "a and q must not be NULL");
      PE_REQUIRE(b.n >= 1 && b.m >= b.n && b.n <= 1024, w + "needs m >= n >= 1 and n <= 1024");
    }
    Ctx& C = *ctx->c;
    dev::set_device(C.device);
    Arena fixed(noalloc_scratch(C.device), NOALLOC_BYTES);
    Rec rec(&C, &fixed);
    rec.set_plain();
    int mm = 0, nn = 0;
    for (int i = 0; i < n_blocks; ++i) {
      mm = std::max(mm, blk[i].m);
      nn = std::max(nn, blk[i].n);
    }
    const bool streaming = Rec::qr_streaming(mm, nn);
    std::vector<QrDesc> ds;
    for (int i = 0; i < n_blocks; ++i) {
      const peps_qr_block& b = blk[i];
      // the streaming kernel's workspace, the only route that uses it
      double* w = streaming ? (double*)fixed.alloc(sizeof(double) * 2 * (size_t)b.m * b.n) : nullptr;
      ds.push_back(QrDesc{b.a, b.a_rs, b.a_cs, b.q, b.q_rs, b.q_cs, b.r, b.r_rs, b.r_cs, w, b.m, b.n});
    }
    rec.qr(ds);
    rec.run(fixed);
  });
}
