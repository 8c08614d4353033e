// gsvd_thin_noalloc: gsvd_thin with its workspace in a fixed device array.
//
// The array is a file-scope __device__ object, so each GPU the library runs on
// holds its own copy from module load until the process ends.  Host code never
// passes the array's name to a kernel (on the host that name is only a stand-in):
// its device address is taken once per device with hipGetSymbolAddress, with
// that device current, and kept in a per-device table.
//
// The calls share the array: two calls that overlap on one GPU (different
// streams, or host threads) race on it.  Nothing in gsvd_thin's kernels relies
// on the workspace's previous contents (every buffer is written before it is
// read, flags are cleared by kernels of the call itself).
#include <hip/hip_runtime.h>

#include <mutex>

#include "api_util.hpp"
#include "gsvd.h"

namespace {

constexpr size_t kScratchBytes = (size_t)GSVD_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// The calling thread's current device's copy of the array (nullptr on failure).
void *scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" {

size_t gsvd_noalloc_max_bytes(void) { return kScratchBytes; }

int gsvd_thin_noalloc(int64_t m, int64_t n, const void *dA, int64_t lda, void *dS, void *dV,
                      int64_t ldv, void *dU, int64_t ldu, int *dInfo, const gsvd_opts *o,
                      void *stream) {
    if (m < 1) return -1;
    if (n < 1 || n > GSVD_MAX_N || n > m) return -2;
    if (dA == nullptr) return -3;
    if (lda < m) return -4;
    if (dS == nullptr) return -5;
    if (dV == nullptr) return -6;
    if (ldv < n) return -7;
    if (int e = gsvd::check_opts(o, 11)) return e;
    if ((o->flags & GSVD_WANT_U) != 0) {
        if (dU == nullptr) return -8;
        if (ldu < m) return -9;
    }
    if (dInfo == nullptr) return -10;
    const size_t need = gsvd_thin_workspace_size(m, n, o);
    if (need == 0 || need > kScratchBytes) return GSVD_ERR_SCRATCH;
    void *work = scratch_ptr();
    if (work == nullptr) return GSVD_ERR_HIP;
    return gsvd_thin(m, n, dA, lda, dS, dV, ldv, dU, ldu, work, kScratchBytes, dInfo, o, stream);
}

}  // extern "C"
