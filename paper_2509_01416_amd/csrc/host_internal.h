// host_internal.h -- host-side state of a tr_context (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.h"
#include "mdpnop.h"

namespace mdp {

struct Ctx;

// Device workspace, grown on demand with hipMalloc; a fixed (external)
// arena never allocates and refuses requests beyond its size.
struct Arena {
    void* base = nullptr;
    size_t cap = 0;
    bool fixed = false;
    bool reserve(Ctx* c, size_t bytes);
};

// Host staging and read-back buffer: pinned memory grown on demand, or a
// fixed buffer that never allocates.
struct PinnedBuf {
    void* ptr = nullptr;
    size_t cap = 0;
    bool fixed = false;
    bool reserve(Ctx* c, size_t bytes);
};

// Host staging area of the no-allocation entry point, allocated with the
// context (ordinary host memory).
constexpr size_t kNoAllocHostBytes = 2u << 20;
// Per-device address of the library's fixed device scratch (nullptr if the
// lookup failed); looked up once per device by noalloc_init.
bool noalloc_init(int device);
void* noalloc_scratch(int device, size_t* bytes);

// Launch plan of the 2-D sweep: D directions per lane, W waves per
// workgroup, per-instance rows per segment R and slices S, LDS block KB.
struct Plan {
    int D = 1, W = 1, KB = 16;
    bool fast = false;   // specialised kernel (R = 64 everywhere, vacuum faces)
    bool p1 = false;     // anisotropic (P1) emission: generic kernel, D = 1
    size_t lds = 0;
    std::vector<int> R, S;
};

struct Setup {
    DirTable dt;
    Plan plan;
    std::vector<InstDesc> inst;
    std::vector<SweepWork> work;
    std::vector<int4> blocks;   // (instance, first cell, reduction slot, -)
    InstDesc* d_inst = nullptr;
    SweepWork* d_work = nullptr;
    int4* d_blocks = nullptr;
    DirTable* d_dt = nullptr;
    double2* d_red = nullptr;
    IterState st{};
    double* d_bal = nullptr;
    int* d_flags = nullptr;
    float* d_samax = nullptr;
    double* d_bpart = nullptr;   // balance partials, 3 per reduction block
    int* d_bar = nullptr;        // persistent iteration: barrier counters (n_inst)
    int* d_err = nullptr;        // persistent iteration: barrier time-out flag
    bool persist = false;        // iterations run as one cooperative launch per chunk
};

struct FnoWork;

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    Arena arena;          // per-call solver workspace
    Arena eig;            // k-eigenvalue workspace (fission source, last iterate, state)
    PinnedBuf pinned;     // staging and flag read-back
    char* noalloc_host = nullptr;   // kNoAllocHostBytes, see tr_solve_noalloc
    int force_D = 0, force_W = 0, force_S = 0, force_R = 0, force_KB = 0;
    bool force_generic = false;   // never use the specialised sweep kernel
    int stop_rule = TR_STOP_CHANGE;   // tr_solve's stopping rule (tr_stop_rule)
    bool sync_checks = false;         // synchronise and check after every HIP step
    bool persistent = false;          // persistent iteration where the plan allows it (opt-in)
    int persist_spin = 1 << 18;       // polls before a persistent barrier wait gives up
    size_t lds_limit = 160 * 1024;  // per-workgroup LDS (gfx950; device property when known)
    int last_sweeps = 0;
    FnoWork* fno = nullptr;   // network workspaces

    // optional kernel timing with HIP events on the context stream
    static constexpr int kProfSlots = 128;
    bool prof = false;
    hipEvent_t ev[kProfSlots][2] = {};
    int ev_kind[kProfSlots] = {};
    int ev_used = 0;
    double prof_ms[4] = {0, 0, 0, 0};   // sweep, combine + finalize, persistent
    long long prof_n[4] = {0, 0, 0, 0};
    bool prof_begin(int kind);      // records the start event; false if full
    void prof_end();
    void prof_collect();            // after a stream synchronisation

    void fail(const char* fmt, ...);
    bool hip_ok(hipError_t e, const char* what);
    void release();
    void release_fno();
    bool setup(int n_inst, const tr_problem* p, const tr_quadrature* q,
               const float* const* phi_init, float* const* phi_out,
               const float* const* emission, Setup* su, bool snapshots = false);
    bool launch_sweep(const Setup& su, int n_inst, const int* done,
                      const int* iter, int use_faces, bool tally = false,
                      const FinArgs* fin = nullptr);
    tr_status scan_fields(const Setup& su, int n_inst, const tr_problem* p,
                          bool need_xs, tr_stats* stats);
    bool si_iterate(const Setup& su, int n_inst, double atol, int norm_kind, int max_iter,
                    int* sweeps, int first_chunk = 4, int* iters_host = nullptr);
    bool si_balance(const Setup& su, int n_inst);
};

size_t align_up(size_t x);
bool build_dirtable(Ctx* c, const tr_quadrature* q, int dim, DirTable* t);
bool check_problems(Ctx* c, int n_inst, const tr_problem* p, bool need_xs);
// true (with the message set) if a problem carries P1 scattering
bool reject_anisotropic(Ctx* c, int n_inst, const tr_problem* p, const char* who);
Plan make_plan(Ctx* c, int n_inst, const tr_problem* p, const DirTable& dt,
               bool p1 = false);

}  // namespace mdp
