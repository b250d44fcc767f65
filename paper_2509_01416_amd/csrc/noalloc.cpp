// noalloc.cpp -- tr_solve_noalloc: the source iteration of tr_solve with
// every device workspace in one fixed, statically sized device array, for
// callers that cannot allocate (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// The array lives in the library's code object: each device the library
// runs on holds its own copy for the life of the process.  Host code never
// uses its name as an address (on the host it is only a stand-in); the
// device address comes from hipGetSymbolAddress, looked up once per device
// with that device current (at context creation) and kept per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host_internal.h"
#include "mdpnop.h"

namespace mdp {

// Largest workspace of one tr_solve_noalloc call: 128 MiB (the 16-problem
// 256 x 256 S16 batch needs about 95 MB).
constexpr size_t kScratchBytes = 128u << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_lock;
static void* g_ptr[kMaxDevices] = {};

bool noalloc_init(int device) {
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> g(g_lock);
    if (g_ptr[device]) return true;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
        (void)hipGetLastError();
        return false;
    }
    g_ptr[device] = p;
    return true;
}

void* noalloc_scratch(int device, size_t* bytes) {
    if (bytes) *bytes = kScratchBytes;
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_lock);
    return g_ptr[device];
}

}  // namespace mdp

using namespace mdp;

extern "C" tr_status tr_solve_noalloc(tr_context* ctx, int32_t n_inst, const tr_problem* p,
                                      const tr_quadrature* q, const float* const* phi_init,
                                      float* const* phi_out, double tol, int32_t max_iter,
                                      tr_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    size_t bytes = 0;
    void* base = noalloc_scratch(c->device, &bytes);
    if (!base || !c->noalloc_host) {
        c->fail("the fixed scratch of device %d is not available", c->device);
        return TR_ERR_HIP;
    }
    // run tr_solve with the fixed scratch and host staging area in place of
    // the context's growable workspaces (fixed: a request beyond them fails
    // in the argument phase, before any launch) and kernel timing off (its
    // events would be created on first use)
    const Arena arena = c->arena;
    const PinnedBuf pinned = c->pinned;
    const bool prof = c->prof;
    c->arena = Arena{base, bytes, true};
    c->pinned = PinnedBuf{c->noalloc_host, kNoAllocHostBytes, true};
    c->prof = false;
    const tr_status s = tr_solve(ctx, n_inst, p, q, phi_init, phi_out, tol, max_iter, stats);
    c->arena = arena;
    c->pinned = pinned;
    c->prof = prof;
    return s;
}
