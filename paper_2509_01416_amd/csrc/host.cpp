// host.cpp -- the C ABI of libmdpnop (see include/mdpnop.h): argument
// checks, quadrature tables, launch planning, workspaces and the source
// iteration driver.  All device work goes to the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mdpnop.h"
#include "common.h"
#include "host_internal.h"

namespace mdp {

bool launch_sweep2d(int D, bool refl, int nwork, int W, int KB,
                    size_t lds_bytes, const InstDesc* insts,
                    const SweepWork* work, const DirTable* dt, const int* done,
                    const int* iter, int use_faces, const FinArgs& fin, hipStream_t s,
                    bool p1);
size_t sweep2d_lds_bytes(int W, int KB, int D, int max_nseg_nx, int max_nx, bool p1);
bool launch_sweep2d_fast(int D, int nwork, int W, int KB, size_t lds_bytes,
                         const InstDesc* insts, const SweepWork* work, const DirTable* dt,
                         const int* done, const int* iter, bool tally, const FinArgs& fin,
                         hipStream_t s);
size_t sweep2d_fast_lds_bytes(int W, int KB, int D, int max_nx);
bool persistent_supported(int D, int W, int KB);
bool persistent_fits(int W, int KB, size_t lds, int nwork, int device);
hipError_t launch_persistent(int W, int KB, size_t lds, int nwork, const InstDesc* insts,
                             const SweepWork* work, const DirTable* dt, const PersistArgs& pa,
                             hipStream_t s);
int sweep2d_max_kb(int W, int R, bool p1);
bool sweep2d_generic_fits(int W, int KB, int R, bool p1);
int sweep2d_fast_max_kb(int W);
int sweep2d_max_w(int D);
void launch_sweep1d(int n_inst, const InstDesc* insts, const DirTable* dt,
                    const int* done, const int* iter, int use_faces, int M,
                    hipStream_t s);
void launch_scan(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                 double* part, int* flags, float* samax, hipStream_t s);
void launch_init(int n_inst, int nblocks, const InstDesc* insts,
                 const int4* blocks, const DirTable* dt, IterState st,
                 const int* skip, hipStream_t s);
void launch_combine(int nblocks, const InstDesc* insts, const int4* blocks,
                    const int* done, double2* red, int mode, int norm_kind,
                    hipStream_t s, const DirTable* dt);
void launch_finalize(int n_inst, const InstDesc* insts, const double2* red,
                     IterState st, double tol, int norm_kind, hipStream_t s);
void launch_balance(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                    const DirTable* dt, const int* iter, double* part, double* bal,
                    hipStream_t s);

// ------------------------------------------------------------ helpers ----

void Ctx::fail(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
}

bool Ctx::hip_ok(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        fail("%s: %s", what, hipGetErrorString(e));
        return false;
    }
    if (sync_checks) {
        // debugging: wait for the work enqueued so far, so that an error of
        // an asynchronous launch is reported at the step that caused it
        hipError_t s = hipStreamSynchronize(stream);
        if (s == hipSuccess) s = hipGetLastError();
        if (s != hipSuccess) {
            fail("%s (synchronous check): %s", what, hipGetErrorString(s));
            return false;
        }
    }
    return true;
}

// Grow-only device arena; sub-allocations are 256-byte aligned.
bool Arena::reserve(Ctx* c, size_t bytes) {
    if (bytes <= cap) return true;
    if (fixed) {
        c->fail("workspace of %zu bytes exceeds the fixed scratch of %zu bytes", bytes, cap);
        return false;
    }
    if (base) { (void)hipFree(base); base = nullptr; cap = 0; }
    size_t want = std::max(bytes, cap * 3 / 2);
    if (hipMalloc(&base, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&base, bytes) != hipSuccess) {
            (void)hipGetLastError();
            base = nullptr;
            c->fail("out of device memory (%zu bytes)", bytes);
            return false;
        }
        want = bytes;
    }
    cap = want;
    return true;
}

bool PinnedBuf::reserve(Ctx* c, size_t bytes) {
    if (bytes <= cap) return true;
    if (fixed) {
        c->fail("host staging of %zu bytes exceeds the fixed buffer of %zu bytes", bytes, cap);
        return false;
    }
    if (ptr) { (void)hipHostFree(ptr); ptr = nullptr; cap = 0; }
    if (hipHostMalloc(&ptr, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
        c->fail("out of pinned host memory (%zu bytes)", bytes);
        return false;
    }
    cap = bytes;
    return true;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// --------------------------------------------------------- quadrature ----

int octant_of(double mu, double eta, int dim) {
    if (dim == 1) return mu > 0 ? 0 : 1;
    if (mu > 0 && eta > 0) return 0;
    if (mu < 0 && eta > 0) return 1;
    if (mu < 0 && eta < 0) return 2;
    return 3;
}

static int find_dir(const tr_quadrature* q, double mu, double eta, int dim) {
    for (int k = 0; k < q->n_dir; ++k) {
        const double de = dim == 2 ? std::fabs(q->eta[k] - eta) : 0.0;
        if (std::fabs(q->mu[k] - mu) < 1e-12 && de < 1e-12) return k;
    }
    return -1;
}

bool build_dirtable(Ctx* c, const tr_quadrature* q, int dim, DirTable* t) {
    if (!q || q->n_dir <= 0 || q->n_dir > kMaxDir || !q->mu || !q->w ||
        (dim == 2 && !q->eta)) {
        c->fail("quadrature: need 1..%d directions with mu, w%s", kMaxDir,
                dim == 2 ? ", eta" : "");
        return false;
    }
    const int M = q->n_dir;
    double sw = 0.0;
    std::memset(t, 0, sizeof(DirTable));
    t->M = M;
    for (int m = 0; m < M; ++m) {
        const double mu = q->mu[m], eta = dim == 2 ? q->eta[m] : 0.0, w = q->w[m];
        if (!std::isfinite(mu) || !std::isfinite(eta) || !std::isfinite(w) ||
            w < 0.0 || mu == 0.0 || (dim == 2 && eta == 0.0) ||
            std::fabs(mu) > 1.0 || std::fabs(eta) > 1.0) {
            c->fail("quadrature: direction %d invalid (mu=%g eta=%g w=%g)", m,
                    mu, eta, w);
            return false;
        }
        sw += w;
        const int o = octant_of(mu, eta, dim);
        t->list[o][t->count[o]++] = m;
        t->amu[m] = (float)std::fabs(mu);
        t->aeta[m] = (float)std::fabs(eta);
        t->mu[m] = (float)mu;
        t->eta[m] = (float)eta;
        t->w[m] = (float)w;
        const int mx = find_dir(q, -mu, eta, dim);
        const int my = dim == 2 ? find_dir(q, mu, -eta, dim) : m;
        if (mx < 0 || my < 0 || std::fabs(q->w[mx] - w) > 1e-12 ||
            std::fabs(q->w[my] - w) > 1e-12) {
            c->fail("quadrature: not reflection symmetric at direction %d", m);
            return false;
        }
        t->mirx[m] = mx;
        t->miry[m] = my;
    }
    if (std::fabs(sw - 1.0) > 1e-12) {
        c->fail("quadrature: weights sum to %.15g, expected 1", sw);
        return false;
    }
    return true;
}

// ---------------------------------------------------------- arguments ----

bool reject_anisotropic(Ctx* c, int n_inst, const tr_problem* p, const char* who) {
    for (int i = 0; i < n_inst; ++i)
        if (p[i].sigma_s1 != nullptr) {
            c->fail("problem %d: %s supports isotropic scattering only (sigma_s1 must be NULL)",
                    i, who);
            return true;
        }
    return false;
}

bool check_problems(Ctx* c, int n_inst, const tr_problem* p, bool need_xs) {
    if (n_inst <= 0 || !p) {
        c->fail("need n_inst > 0 problems");
        return false;
    }
    const int dim = p[0].dim;
    for (int i = 0; i < n_inst; ++i) {
        const tr_problem& P = p[i];
        if (P.dim != 1 && P.dim != 2) {
            c->fail("problem %d: dim must be 1 or 2", i);
            return false;
        }
        if (P.dim != dim) {
            c->fail("problem %d: all problems of a call must share dim", i);
            return false;
        }
        const int ny = P.dim == 1 ? 1 : P.ny;
        if (P.nx <= 0 || ny <= 0 || (int64_t)P.nx * ny > (1LL << 30)) {
            c->fail("problem %d: bad grid %d x %d", i, P.nx, P.ny);
            return false;
        }
        if (P.dim == 2 && P.ny <= 0) {
            c->fail("problem %d: ny must be positive", i);
            return false;
        }
        if (!(P.lx > 0.0) || !std::isfinite(P.lx) ||
            (P.dim == 2 && (!(P.ly > 0.0) || !std::isfinite(P.ly)))) {
            c->fail("problem %d: extents must be positive and finite", i);
            return false;
        }
        if (!P.sigma_t || (need_xs && (!P.sigma_s || !P.source))) {
            c->fail("problem %d: missing field pointer", i);
            return false;
        }
        const int nb = P.dim == 1 ? 2 : 4;
        for (int f = 0; f < nb; ++f)
            if (P.bc[f] != TR_BC_VACUUM && P.bc[f] != TR_BC_REFLECTIVE) {
                c->fail("problem %d: bc[%d] = %d is not a tr_bc", i, f, P.bc[f]);
                return false;
            }
    }
    return true;
}

}  // namespace mdp

using namespace mdp;

// ===================================================================== ABI

extern "C" tr_status tr_context_create(tr_context** ctx, void* hip_stream) {
    if (!ctx) return TR_ERR_INVALID_ARG;
    *ctx = nullptr;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return TR_ERR_HIP;
    }
    Ctx* c = new (std::nothrow) Ctx();
    if (!c) return TR_ERR_OOM;
    c->device = dev;
    {
        const char* env = std::getenv("MDPNOP_SYNC_CHECKS");
        c->sync_checks = env != nullptr && env[0] != '\0' && env[0] != '0';
    }
    c->noalloc_host = new (std::nothrow) char[kNoAllocHostBytes];
    if (!c->noalloc_host) {
        delete c;
        return TR_ERR_OOM;
    }
    // the fixed scratch of tr_solve_noalloc: its address on this device
    if (!noalloc_init(dev)) {
        delete[] c->noalloc_host;
        delete c;
        return TR_ERR_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.sharedMemPerBlock > 0)
        c->lds_limit = prop.sharedMemPerBlock;
    else
        (void)hipGetLastError();
    c->stream = (hipStream_t)hip_stream;
    *ctx = reinterpret_cast<tr_context*>(c);
    return TR_OK;
}

extern "C" void tr_context_destroy(tr_context* ctx) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    c->release();
    delete[] c->noalloc_host;
    delete c;
}

extern "C" const char* tr_last_error(const tr_context* ctx) {
    const Ctx* c = reinterpret_cast<const Ctx*>(ctx);
    return c ? c->err.c_str() : "null context";
}

bool Ctx::prof_begin(int kind) {
    if (!prof || ev_used >= kProfSlots) return false;
    hipEvent_t* e = ev[ev_used];
    if (!e[0]) {
        if (hipEventCreate(&e[0]) != hipSuccess || hipEventCreate(&e[1]) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
    }
    ev_kind[ev_used] = kind;
    (void)hipEventRecord(e[0], stream);
    return true;
}

void Ctx::prof_end() { (void)hipEventRecord(ev[ev_used++][1], stream); }

void Ctx::prof_collect() {
    for (int i = 0; i < ev_used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[i][0], ev[i][1]) == hipSuccess) {
            prof_ms[ev_kind[i]] += ms;
            prof_n[ev_kind[i]] += 1;
        } else {
            (void)hipGetLastError();
        }
    }
    ev_used = 0;
}

void Ctx::release() {
    for (auto& e : ev) {
        if (e[0]) (void)hipEventDestroy(e[0]);
        if (e[1]) (void)hipEventDestroy(e[1]);
        e[0] = e[1] = nullptr;
    }
    for (Arena* a : {&arena, &eig}) {
        if (a->base) (void)hipFree(a->base);
        a->base = nullptr;
        a->cap = 0;
    }
    if (pinned.ptr) (void)hipHostFree(pinned.ptr);
    pinned.ptr = nullptr;
    pinned.cap = 0;
    release_fno();
}

// --------------------------------------------------------------- plan ----

namespace mdp {

// Launch planning for the 2-D sweep.  A segment of R lanes streams through
// ceil(ny/R) row blocks of nx cells: T = ceil(ny/R)*nx + R - 1 steps, and an
// octant of nd directions needs v = ceil(nd*R/(64*D)) waves.  The plan picks
// R per instance to minimise the modelled time
//     max( sum_i 4 v_i T_i / NW , max_i T_i )
// (NW = waves the chip keeps busy), trying the widest feasible R for every
// instance (latency-bound batches) and the R with the fewest lane-steps
// 4 v T per instance (throughput-bound batches).  W waves per workgroup and
// S slices per octant then give at least one workgroup per CU (generic
// kernel) or the shortest step time (specialised kernel, see below).
namespace {
constexpr double kBusyWaves = 2048.0;   // ~2 waves per SIMD on 256 CUs
constexpr int kCUs = 256;

long long seg_steps(int nx, int ny, int R) {
    return (long long)((ny + R - 1) / R) * nx + R - 1;
}
int oct_waves(int nd, int R, int D) {
    const int per = (64 / R) * D;
    return (nd + per - 1) / per;
}
}  // namespace

namespace {
Plan plan_impl(Ctx* c, int n_inst, const tr_problem* p, const DirTable& dt, bool p1,
               bool try_fast) {
    Plan pl;
    int nd = 0;
    for (int o = 0; o < 4; ++o) nd = std::max(nd, dt.count[o]);
    // anisotropic (P1) emission: the generic kernel with one direction per lane
    pl.p1 = p1;
    pl.D = p1 ? 1 : (c->force_D > 0 ? c->force_D : 1);
    pl.R.assign(n_inst, 1);
    // grids the specialised kernel takes (block size aside): vacuum faces,
    // 64-row segments (a ragged last row block is fine), and either several
    // row blocks with nx >= 63 + KB or one row block with nx >= ny - 1
    bool fast = try_fast && !c->force_generic && pl.D <= 4 && !p1 &&
                (c->force_R <= 0 || c->force_R == 64);
    int nxmin = 1 << 30, nxall = 1 << 30;
    for (int i = 0; i < n_inst && fast; ++i) {
        for (int f = 0; f < 4; ++f) fast = fast && p[i].bc[f] == TR_BC_VACUUM;
        nxall = std::min(nxall, p[i].nx);
        if (p[i].ny > 64) nxmin = std::min(nxmin, p[i].nx);
        else fast = fast && p[i].nx >= p[i].ny - 1;
    }
    fast = fast && nxall >= 2 && nxmin >= 65;
    auto model = [&](const std::vector<int>& Rs) {
        double work = 0.0, tmax = 0.0;
        for (int i = 0; i < n_inst; ++i) {
            const double T = (double)seg_steps(p[i].nx, p[i].ny, Rs[i]);
            work += 4.0 * oct_waves(nd, Rs[i], pl.D) * T;
            tmax = std::max(tmax, T);
        }
        return std::max(work / kBusyWaves, tmax);
    };
    // R: a power of two <= min(64, nx) that divides ny (the sweep kernel's
    // ring writer is the last lane of each segment)
    auto feasible = [&](int i, int R) { return R <= p[i].nx && p[i].ny % R == 0; };
    std::vector<int> wide(n_inst), lean(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        int rw = 1;
        while (rw * 2 <= 64 && feasible(i, rw * 2)) rw *= 2;
        wide[i] = rw;
        double best = 1e300;
        int rb = rw;
        for (int R = rw; R >= 1; R >>= 1) {
            if (!feasible(i, R)) continue;
            const double cost = (double)oct_waves(nd, R, pl.D) * seg_steps(p[i].nx, p[i].ny, R);
            if (cost < best * 0.999) { best = cost; rb = R; }
        }
        lean[i] = rb;
    }
    pl.R = model(wide) <= model(lean) ? wide : lean;
    if (c->force_R > 0)
        for (int i = 0; i < n_inst; ++i)
            if (feasible(i, c->force_R)) pl.R[i] = c->force_R;
    if (fast) pl.R.assign(n_inst, 64);
    // W and S: the largest W (fewest partial planes) that still yields at
    // least one workgroup per CU (or every wave in its own slice)
    int vmax = 1;
    long long vsum = 0;
    for (int i = 0; i < n_inst; ++i) {
        const int v = oct_waves(nd, pl.R[i], pl.D);
        vmax = std::max(vmax, v);
        vsum += 4LL * v;
    }
    const long long want = std::min<long long>(kCUs, vsum);
    const int wcap = sweep2d_max_w(pl.D);
    int W = std::min(wcap, vmax);
    bool step_rule = false;   // W set for the specialised kernel's step time
    if (c->force_W > 0) {
        W = std::min(c->force_W, wcap);
    } else if (fast && pl.D == 1 && c->force_S <= 0) {
        // specialised kernel: an instance's chain takes T steps whatever
        // the number of busy CUs, so a batch too small to fill the chip is
        // bound by the step time, which is shortest near one wave per SIMD
        // (W = 4, the fewest waves that keep 16-step blocks, idle waves
        // included where an octant has fewer directions).  Take the most
        // slices per octant, up to ceil(nd/4) and at most 6 (each slice
        // adds 4 partial planes to the iteration's sum: on 128^2 S16 grids
        // 8 slices of 5 waves cost 7 % more per iteration than 6 of 6),
        // whose workgroups still find a CU each on the instance's XCD
        // (32 CUs; instances spread over the 8 XCDs), and one slice once
        // the batch fills it.
        const int per_xcd = (n_inst + kXcds - 1) / kXcds;
        const int smax = std::min(6, (nd + 3) / 4);
        int S = 1;
        for (int s = 2; s <= smax && 4LL * per_xcd * s <= kCUs / kXcds; ++s) S = s;
        W = std::min(wcap, std::max(4, (nd + S - 1) / S));
        step_rule = true;
        // a wide grid's LDS ring (nx values per wave) may allow fewer waves
        int nxw = 1;
        for (int i = 0; i < n_inst; ++i) nxw = std::max(nxw, p[i].nx);
        while (W > 1 && sweep2d_fast_lds_bytes(W, 2, pl.D, nxw) > c->lds_limit) --W;
    } else {
        for (; W > 1; --W) {
            long long wgs = 0;
            for (int i = 0; i < n_inst; ++i) {
                const int v = oct_waves(nd, pl.R[i], pl.D);
                wgs += 4LL * ((v + W - 1) / W);
            }
            if (wgs >= want) break;
        }
    }
    pl.S.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const int cap = W * (64 / pl.R[i]) * pl.D;
        pl.S[i] = c->force_S > 0 ? std::max(c->force_S, (nd + cap - 1) / cap)
                                 : std::max(1, (nd + cap - 1) / cap);
    }
    if (c->force_W <= 0 && !step_rule) {   // same slice counts, fewest idle waves
        int wmin = 1;
        for (int i = 0; i < n_inst; ++i) {
            const int v = oct_waves(nd, pl.R[i], pl.D);
            wmin = std::max(wmin, (v + pl.S[i] - 1) / pl.S[i]);
        }
        W = wmin;
    }
    pl.W = W;
    int mx = 0, Rmax = 1, nxmax = 1;
    for (int i = 0; i < n_inst; ++i) {
        mx = std::max(mx, (64 / pl.R[i]) * p[i].nx);
        Rmax = std::max(Rmax, pl.R[i]);
        nxmax = std::max(nxmax, p[i].nx);
    }
    // the specialised kernel's block size: KB <= nx everywhere (a lane
    // restarts at most once per block) and nx >= 63 + KB wherever a grid
    // has more than one row block (lane 0's ring column is then always
    // written in an earlier block); otherwise the generic kernel with its
    // own segment heights
    const int kb0 = std::min(c->force_KB > 0 ? c->force_KB : 16, sweep2d_max_kb(W, Rmax, p1));
    if (fast) {
        int kb = std::min(c->force_KB > 0 ? c->force_KB : 16, sweep2d_fast_max_kb(W));
        auto kb_ok = [&](int k) {
            return nxmin >= 63 + k && k <= nxall &&
                   sweep2d_fast_lds_bytes(W, k, pl.D, nxmax) <= c->lds_limit;
        };
        while (kb > 2 && !kb_ok(kb)) kb /= 2;
        if (kb >= 2 && kb_ok(kb)) {
            pl.fast = true;
            pl.KB = kb;
            pl.lds = sweep2d_fast_lds_bytes(W, kb, pl.D, nxmax);
            return pl;
        }
        return plan_impl(c, n_inst, p, dt, p1, false);
    }
    pl.fast = false;
    pl.KB = kb0;
    while (pl.KB > 2 && sweep2d_lds_bytes(W, pl.KB, pl.D, mx, nxmax, p1) > c->lds_limit)
        pl.KB /= 2;
    pl.KB = std::max(pl.KB, 2);
    pl.lds = sweep2d_lds_bytes(W, pl.KB, pl.D, mx, nxmax, p1);
    return pl;
}
}  // namespace

Plan make_plan(Ctx* c, int n_inst, const tr_problem* p, const DirTable& dt, bool p1) {
    return plan_impl(c, n_inst, p, dt, p1, true);
}

// Builds descriptors and workspaces for n_inst problems.  emission != nullptr
// selects a bare sweep (Q = caller emission, phi = phi_out).
bool Ctx::setup(int n_inst, const tr_problem* p, const tr_quadrature* q,
                const float* const* phi_init, float* const* phi_out,
                const float* const* emission, Setup* su, bool snapshots) {
    const int dim = p[0].dim;
    if (!build_dirtable(this, q, dim, &su->dt)) return false;
    const int M = su->dt.M;
    // linearly anisotropic scattering in a source iteration (a bare sweep
    // has no current to feed it): every problem of the launch then carries
    // the emission fields and current planes
    bool p1 = false;
    if (!emission)
        for (int i = 0; i < n_inst; ++i) p1 = p1 || p[i].sigma_s1 != nullptr;
    if (dim == 2) {
        for (int o = 0; o < 4; ++o)
            if (su->dt.count[o] != su->dt.count[0]) {
                fail("quadrature: octants hold different direction counts");
                return false;
            }
        su->plan = make_plan(this, n_inst, p, su->dt, p1);
        if (su->plan.lds > lds_limit) {
            fail("grid too wide for the sweep's LDS ring (nx=%d)", p[0].nx);
            return false;
        }
        if (!su->plan.fast)
            for (int i = 0; i < n_inst; ++i)
                if (!sweep2d_generic_fits(su->plan.W, su->plan.KB, su->plan.R[i], p1)) {
                    fail("internal: launch shape W=%d KB=%d R=%d exceeds the sweep's "
                         "staging slots", su->plan.W, su->plan.KB, su->plan.R[i]);
                    return false;
                }
    }
    su->inst.resize(n_inst);
    su->blocks.clear();
    su->work.clear();
    size_t off = 0;
    std::vector<size_t> offQ(n_inst), offP(n_inst), offF(n_inst), offS(n_inst), offE(n_inst),
        offJ(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const tr_problem& P = p[i];
        InstDesc& d = su->inst[i];
        std::memset(&d, 0, sizeof d);
        d.dim = dim;
        d.nx = P.nx;
        d.ny = dim == 1 ? 1 : P.ny;
        d.nf = std::max(d.nx, d.ny);
        d.cells = d.nx * d.ny;
        d.dx = P.lx / P.nx;
        d.dy = dim == 1 ? 1.0 : P.ly / P.ny;
        d.inv_dx = (float)(1.0 / d.dx);
        d.inv_dy = (float)(1.0 / d.dy);
        for (int f = 0; f < 4; ++f) d.bc[f] = (dim == 1 && f >= 2) ? 0 : P.bc[f];
        d.st = P.sigma_t;
        d.ss = P.sigma_s;
        d.q = P.source;
        d.phi = phi_out[i];
        d.phi_init = phi_init ? phi_init[i] : nullptr;
        if (dim == 2) {
            d.R = su->plan.R[i];
            d.S = su->plan.S[i];
            d.P = 4 * d.S;
            for (int o = 0; o < 4; ++o)
                for (int s = 0; s < d.S; ++s) su->work.push_back({i, o, s, 0});
        } else {
            d.R = 1;
            d.S = 1;
            d.P = M;
        }
        d.red0 = (int)su->blocks.size();
        for (int c0 = 0; c0 < d.cells; c0 += kCombineChunk)
            su->blocks.push_back(make_int4(i, c0, (int)su->blocks.size(), 0));
        d.nred = (int)su->blocks.size() - d.red0;
        if (!emission) {
            offQ[i] = off;
            off += align_up(sizeof(float) * d.cells);
        }
        offP[i] = off;
        off += align_up(sizeof(float) * (size_t)d.P * d.cells);
        offF[i] = off;
        off += align_up(sizeof(float) * (dim == 1 ? (size_t)4 * M
                                                   : (size_t)8 * d.nf * M));
        if (snapshots) {
            offS[i] = off;
            off += align_up(sizeof(float) * d.cells);
        }
        if (p1) {
            d.ss1 = P.sigma_s1;
            offE[i] = off;   // Ex (and Ey in 2-D)
            off += align_up(sizeof(float) * (size_t)(dim == 1 ? 1 : 2) * d.cells);
            if (dim == 2) {
                offJ[i] = off;
                off += align_up(sizeof(float) * (size_t)2 * d.P * d.cells);
            }
        }
    }
    // XCD-aware order: workgroup b of a launch runs on XCD b % kXcds, so
    // every instance is given one XCD (balanced by work) and its sweep
    // workgroups and combine blocks are placed at indices of that XCD; the
    // instance's fields and partial planes then stay in that XCD's L2.
    // Queues are padded with no-op entries (instance -1) to keep alignment.
    {
        std::vector<int> bucket(n_inst);
        std::vector<double> load(kXcds, 0.0);
        std::vector<int> order(n_inst);
        for (int i = 0; i < n_inst; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return su->inst[x].cells > su->inst[y].cells;
        });
        for (int i : order) {
            int bx = 0;
            for (int x = 1; x < kXcds; ++x)
                if (load[x] < load[bx]) bx = x;
            bucket[i] = bx;
            load[bx] += (double)su->inst[i].cells * su->inst[i].P;
        }
        auto interleave = [&](auto& items, auto bucket_of, auto make_noop) {
            using T = typename std::decay<decltype(items[0])>::type;
            std::vector<std::vector<T>> q(kXcds);
            for (const T& it : items) q[bucket_of(it)].push_back(it);
            size_t mx = 0;
            for (auto& v : q) mx = std::max(mx, v.size());
            std::vector<T> out;
            out.reserve(mx * kXcds);
            for (size_t r = 0; r < mx; ++r)
                for (int x = 0; x < kXcds; ++x)
                    out.push_back(r < q[x].size() ? q[x][r] : make_noop());
            // trailing no-ops are not launched
            while (!out.empty() && (&out.back() != nullptr) && bucket_of(out.back()) < 0)
                out.pop_back();
            items.swap(out);
        };
        // within an XCD's queue the longest chains (ceil(ny/R) nx + R - 1
        // steps) go first: workgroups are handed to the XCD's CUs in turn,
        // so every CU gets a share of the long ones and none starts one last
        if (dim == 2) {
            auto chain = [&](const SweepWork& w) {
                const InstDesc& d = su->inst[w.inst];
                return (long long)((d.ny + d.R - 1) / d.R) * d.nx + d.R - 1;
            };
            std::stable_sort(su->work.begin(), su->work.end(),
                             [&](const SweepWork& x, const SweepWork& y) {
                                 return chain(x) > chain(y);
                             });
        }
        if (!su->work.empty())
            interleave(su->work,
                       [&](const SweepWork& w) { return w.inst < 0 ? -1 : bucket[w.inst]; },
                       []() { return SweepWork{-1, 0, 0, 0}; });
        interleave(su->blocks,
                   [&](const int4& b) { return b.x < 0 ? -1 : bucket[b.x]; },
                   []() { return make_int4(-1, 0, 0, 0); });
    }
    // fixed-size tables after the per-instance workspaces
    size_t nslots = 0;
    for (const InstDesc& d : su->inst) nslots += d.nred;
    const size_t oInst = off;
    off += align_up(sizeof(InstDesc) * n_inst);
    const size_t oWork = off;
    off += align_up(sizeof(SweepWork) * std::max<size_t>(1, su->work.size()));
    const size_t oBlk = off;
    off += align_up(sizeof(int4) * su->blocks.size());
    const size_t oDt = off;
    off += align_up(sizeof(DirTable));
    const size_t oRed = off;
    off += align_up(sizeof(double2) * nslots);
    const size_t oDone = off;
    off += align_up(sizeof(int) * n_inst);
    const size_t oIter = off;
    off += align_up(sizeof(int) * n_inst);
    const size_t oStat = off;
    off += align_up(sizeof(int) * n_inst);
    const size_t oRes = off;
    off += align_up(sizeof(double) * n_inst);
    const size_t oRh = off;
    off += align_up(sizeof(double) * 2 * n_inst);
    const size_t oBal = off;
    off += align_up(sizeof(double) * 3 * n_inst);
    const size_t oFlag = off;
    off += align_up(sizeof(int) * n_inst);
    const size_t oSa = off;
    off += align_up(sizeof(float) * n_inst);
    const size_t oBpart = off;
    off += align_up(sizeof(double) * 3 * std::max<size_t>(1, nslots));
    const size_t oBar = off;
    off += align_up(sizeof(int) * (n_inst + 1));
    if (!arena.reserve(this, off)) return false;
    char* b = (char*)arena.base;
    for (int i = 0; i < n_inst; ++i) {
        InstDesc& d = su->inst[i];
        d.Q = emission ? const_cast<float*>(emission[i]) : (float*)(b + offQ[i]);
        d.part = (float*)(b + offP[i]);
        d.face = (float*)(b + offF[i]);
        d.snap = snapshots ? (float*)(b + offS[i]) : nullptr;
        d.Ex = p1 ? (float*)(b + offE[i]) : nullptr;
        d.Ey = p1 && d.dim == 2 ? d.Ex + d.cells : nullptr;
        d.partJ = p1 && d.dim == 2 ? (float*)(b + offJ[i]) : nullptr;
    }
    su->d_inst = (InstDesc*)(b + oInst);
    su->d_work = (SweepWork*)(b + oWork);
    su->d_blocks = (int4*)(b + oBlk);
    su->d_dt = (DirTable*)(b + oDt);
    su->d_red = (double2*)(b + oRed);
    su->st.done = (int*)(b + oDone);
    su->st.iter = (int*)(b + oIter);
    su->st.status = (int*)(b + oStat);
    su->st.resid = (double*)(b + oRes);
    su->st.rhist = (double*)(b + oRh);
    su->d_bal = (double*)(b + oBal);
    su->d_flags = (int*)(b + oFlag);
    su->d_samax = (float*)(b + oSa);
    su->d_bpart = (double*)(b + oBpart);
    su->d_bar = (int*)(b + oBar);
    su->d_err = su->d_bar + n_inst;
    // source iterations as one cooperative launch per chunk: the specialised
    // sweep's common shapes, when every workgroup of the launch is resident
    su->persist = persistent && dim == 2 && !emission && !p1 && su->plan.fast &&
                  persistent_supported(su->plan.D, su->plan.W, su->plan.KB) &&
                  persistent_fits(su->plan.W, su->plan.KB, su->plan.lds, (int)su->work.size(),
                                  device);
    // stage the tables through pinned memory
    const size_t hsz = oRed - oInst;
    if (!pinned.reserve(this, hsz + 4096 + (size_t)n_inst * 64)) return false;
    if (!hip_ok(hipStreamSynchronize(stream), "sync")) return false;
    char* h = (char*)pinned.ptr;
    std::memcpy(h + (oInst - oInst), su->inst.data(), sizeof(InstDesc) * n_inst);
    if (!su->work.empty())
        std::memcpy(h + (oWork - oInst), su->work.data(),
                    sizeof(SweepWork) * su->work.size());
    std::memcpy(h + (oBlk - oInst), su->blocks.data(),
                sizeof(int4) * su->blocks.size());
    std::memcpy(h + (oDt - oInst), &su->dt, sizeof(DirTable));
    if (!hip_ok(hipMemcpyAsync(b + oInst, h, hsz, hipMemcpyHostToDevice, stream),
                "table upload"))
        return false;
    return true;
}

bool Ctx::launch_sweep(const Setup& su, int n_inst, const int* done,
                       const int* iter, int use_faces, bool tally, const FinArgs* fin) {
    FinArgs none{};
    const FinArgs& fa = fin ? *fin : none;
    if (su.inst[0].dim == 1) {
        launch_sweep1d(n_inst, su.d_inst, su.d_dt, done, iter, use_faces, su.dt.M,
                       stream);
    } else {
        bool refl = false;
        for (const InstDesc& d : su.inst)
            for (int f = 0; f < 4; ++f) refl |= d.bc[f] == TR_BC_REFLECTIVE;
        const bool ok =
            su.plan.fast
                ? launch_sweep2d_fast(su.plan.D, (int)su.work.size(), su.plan.W, su.plan.KB,
                                      su.plan.lds, su.d_inst, su.d_work, su.d_dt, done, iter,
                                      tally, fa, stream)
                : launch_sweep2d(su.plan.D, refl && use_faces, (int)su.work.size(),
                                 su.plan.W, su.plan.KB, su.plan.lds, su.d_inst, su.d_work,
                                 su.d_dt, done, iter, use_faces, fa, stream, su.plan.p1);
        if (!ok) {
            fail("unsupported directions-per-lane D=%d", su.plan.D);
            return false;
        }
    }
    return hip_ok(hipGetLastError(), "sweep launch");
}

// Source iteration from the state launch_init left: sweeps in chunks of
// first_chunk (default 4), then doubling up to 64, between read-backs of the
// per-instance done flags, until every instance is done or max_iter sweeps
// have run.  The convergence test runs after every sweep whatever the chunk
// size: sweeps past an instance's convergence leave at once, so the chunking
// changes no result.  iters_host (pinned, optional) receives the
// per-instance sweep counts with the last read-back.
bool Ctx::si_iterate(const Setup& su, int n_inst, double atol, int norm_kind, int max_iter,
                     int* sweeps, int first_chunk, int* iters_host) {
    int* hdone = (int*)pinned.ptr;
    // the barrier time-out flag reads back into the last bytes of the
    // staging buffer (callers keep their own arrays at its start)
    int* herr = (int*)((char*)pinned.ptr + pinned.cap - 64);
    int done_iters = 0, chunk = std::min(std::max(first_chunk, 1), 64);
    const bool fused_fin = su.inst[0].dim == 2;
    bool all = false;
    if (su.persist &&
        !hip_ok(hipMemsetAsync(su.d_bar, 0, sizeof(int) * (n_inst + 1), stream), "memset"))
        return false;
    while (done_iters < max_iter && !all) {
        const int k = std::min(chunk, max_iter - done_iters);
        if (su.persist) {
            // k iterations (sweep, combine, test) in one cooperative launch
            const PersistArgs pa{su.d_bar, su.d_err, persist_spin, done_iters, k, norm_kind,
                                 atol, su.d_red, su.st};
            const bool p2 = prof_begin(2);
            if (!hip_ok(launch_persistent(su.plan.W, su.plan.KB, su.plan.lds,
                                          (int)su.work.size(), su.d_inst, su.d_work, su.d_dt,
                                          pa, stream), "persistent launch"))
                return false;
            if (p2) prof_end();
        }
        for (int it = 0; it < k && !su.persist; ++it) {
            // 2-D: the convergence test of iteration it - 1 runs in the
            // prologue of sweep it (FinArgs); the chunk's last iteration is
            // tested by the finalize kernel before the flags are read back
            const FinArgs fin{su.d_red, su.st, atol, norm_kind, fused_fin && it > 0 ? 1 : 0,
                              done_iters + it};
            const bool p0 = prof_begin(0);
            if (!launch_sweep(su, n_inst, su.st.done, su.st.iter, 1, false, &fin)) return false;
            if (p0) prof_end();
            const bool p1 = prof_begin(1);
            // the error-bound rule measures the change against the snapshot
            // on its tested iterations (every kStopStride-th) only
            const int l = done_iters + it + 1;
            const int mode = norm_kind != 2 ? 0 : (l % kStopStride == 0 ? 2 : 3);
            launch_combine((int)su.blocks.size(), su.d_inst, su.d_blocks, su.st.done,
                           su.d_red, mode, norm_kind, stream, su.d_dt);
            if (!fused_fin || it + 1 == k)
                launch_finalize(n_inst, su.d_inst, su.d_red, su.st, atol, norm_kind, stream);
            if (p1) prof_end();
        }
        if (!hip_ok(hipGetLastError(), "iteration launch")) return false;
        done_iters += k;
        if (!hip_ok(hipMemcpyAsync(hdone, su.st.done, sizeof(int) * n_inst,
                                   hipMemcpyDeviceToHost, stream), "flag copy") ||
            (su.persist && !hip_ok(hipMemcpyAsync(herr, su.d_err, sizeof(int),
                                                  hipMemcpyDeviceToHost, stream), "flag copy")) ||
            (iters_host && !hip_ok(hipMemcpyAsync(iters_host, su.st.iter, sizeof(int) * n_inst,
                                                  hipMemcpyDeviceToHost, stream), "copy")) ||
            !hip_ok(hipStreamSynchronize(stream), "sync"))
            return false;
        prof_collect();
        if (su.persist && *herr) {
            fail("persistent iteration: an instance barrier wait timed out");
            return false;
        }
        all = true;
        for (int i = 0; i < n_inst; ++i) all &= hdone[i] != 0;
        chunk = std::min(chunk * 2, 64);
    }
    if (sweeps) *sweeps = done_iters;
    return true;
}

// Particle balance of the last sweep into su.d_bal.  The specialised sweep
// stores no boundary faces while iterating (vacuum inflow reads none): one
// more sweep of the final emission tallies them, into the current face
// parity, without touching the iterate.
bool Ctx::si_balance(const Setup& su, int n_inst) {
    if (su.inst[0].dim == 2 && su.plan.fast &&
        !launch_sweep(su, n_inst, nullptr, su.st.iter, 1, true))
        return false;
    launch_balance(n_inst, (int)su.blocks.size(), su.d_inst, su.d_blocks, su.d_dt, su.st.iter,
                   su.d_bpart, su.d_bal, stream);
    return hip_ok(hipGetLastError(), "balance launch");
}

// Field checks on the device: non-finite values, cross-section ranges, and a
// singular system (no absorption anywhere and no vacuum face).
tr_status Ctx::scan_fields(const Setup& su, int n_inst, const tr_problem* p,
                           bool need_xs, tr_stats* stats) {
    (void)need_xs;
    launch_scan(n_inst, (int)su.blocks.size(), su.d_inst, su.d_blocks, su.d_bpart, su.d_flags,
                su.d_samax, stream);
    if (!hip_ok(hipGetLastError(), "scan launch")) return TR_ERR_HIP;
    int* hf = (int*)pinned.ptr;
    float* hs = (float*)((char*)pinned.ptr + align_up(sizeof(int) * n_inst));
    if (!hip_ok(hipMemcpyAsync(hf, su.d_flags, sizeof(int) * n_inst,
                               hipMemcpyDeviceToHost, stream), "flag copy") ||
        !hip_ok(hipMemcpyAsync(hs, su.d_samax, sizeof(float) * n_inst,
                               hipMemcpyDeviceToHost, stream), "flag copy") ||
        !hip_ok(hipStreamSynchronize(stream), "sync"))
        return TR_ERR_HIP;
    tr_status worst = TR_OK;
    for (int i = 0; i < n_inst; ++i) {
        tr_status s = TR_OK;
        if (hf[i] & 1) {
            s = TR_ERR_NONFINITE;
            fail("problem %d: non-finite field value", i);
        } else if (hf[i] & 2) {
            s = TR_ERR_INVALID_ARG;
            fail("problem %d: need sigma_t > 0 and 0 <= sigma_s <= sigma_t", i);
        } else if (hs[i] <= 0.f) {
            const int nb = p[i].dim == 1 ? 2 : 4;
            bool vac = false;
            for (int f = 0; f < nb; ++f) vac |= p[i].bc[f] == TR_BC_VACUUM;
            if (!vac) {
                s = TR_ERR_INVALID_ARG;
                fail("problem %d: no absorption and no vacuum face (singular)", i);
            }
        }
        if (stats) stats[i].status = s;
        if (s < worst) worst = s;
    }
    return worst;
}

}  // namespace mdp

extern "C" tr_status tr_sweep(tr_context* ctx, int32_t n_inst, const tr_problem* p,
                              const tr_quadrature* q,
                              const float* const* emission,
                              float* const* phi_out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!check_problems(c, n_inst, p, false)) return TR_ERR_INVALID_ARG;
    if (!emission || !phi_out) {
        c->fail("emission and phi_out are required");
        return TR_ERR_INVALID_ARG;
    }
    for (int i = 0; i < n_inst; ++i)
        if (!emission[i] || !phi_out[i]) {
            c->fail("problem %d: null emission or phi_out", i);
            return TR_ERR_INVALID_ARG;
        }
    Setup su;
    if (!c->setup(n_inst, p, q, nullptr, phi_out, emission, &su))
        return c->err.rfind("out of", 0) == 0 ? TR_ERR_OOM : TR_ERR_INVALID_ARG;
    if (!c->launch_sweep(su, n_inst, nullptr, nullptr, 0)) return TR_ERR_HIP;
    launch_combine((int)su.blocks.size(), su.d_inst, su.d_blocks, nullptr,
                   su.d_red, 1, 0, c->stream, su.d_dt);
    if (!c->hip_ok(hipGetLastError(), "combine launch")) return TR_ERR_HIP;
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "sync")) return TR_ERR_HIP;
    return TR_OK;
}

extern "C" tr_status tr_solve(tr_context* ctx, int32_t n_inst, const tr_problem* p,
                              const tr_quadrature* q, const float* const* phi_init,
                              float* const* phi_out, double tol, int32_t max_iter,
                              tr_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!check_problems(c, n_inst, p, true)) return TR_ERR_INVALID_ARG;
    if (!phi_out || max_iter <= 0 || !std::isfinite(tol) || tol == 0.0) {
        c->fail("need phi_out, max_iter > 0 and a finite non-zero tol");
        return TR_ERR_INVALID_ARG;
    }
    for (int i = 0; i < n_inst; ++i)
        if (!phi_out[i]) {
            c->fail("problem %d: null phi_out", i);
            return TR_ERR_INVALID_ARG;
        }
    if (c->stop_rule == TR_STOP_ERROR_BOUND && tol < 0) {
        c->fail("the error-bound stopping rule needs tol > 0");
        return TR_ERR_INVALID_ARG;
    }
    const int norm_kind = c->stop_rule == TR_STOP_ERROR_BOUND ? 2 : (tol < 0 ? 1 : 0);
    const double atol = std::fabs(tol);
    Setup su;
    if (!c->setup(n_inst, p, q, phi_init, phi_out, nullptr, &su, norm_kind == 2))
        return c->err.rfind("out of", 0) == 0 ? TR_ERR_OOM : TR_ERR_INVALID_ARG;
    if (stats)
        for (int i = 0; i < n_inst; ++i) stats[i] = tr_stats{0, 0, 0.0, 0.0, 0.0};
    tr_status s0 = c->scan_fields(su, n_inst, p, true, stats);
    if (s0 < 0) return s0;
    launch_init(n_inst, (int)su.blocks.size(), su.d_inst, su.d_blocks, su.d_dt,
                su.st, nullptr, c->stream);
    if (!c->hip_ok(hipGetLastError(), "init launch")) return TR_ERR_HIP;
    int done_iters = 0;
    if (!c->si_iterate(su, n_inst, atol, norm_kind, max_iter, &done_iters) ||
        !c->si_balance(su, n_inst))
        return TR_ERR_HIP;
    // read back iteration state
    if (!c->pinned.reserve(c, 2 * align_up(sizeof(int) * n_inst) +
                                   align_up(sizeof(double) * n_inst) +
                                   align_up(sizeof(double) * 3 * n_inst)))
        return TR_ERR_OOM;
    char* h = (char*)c->pinned.ptr;
    int* hit = (int*)h;
    int* hst = (int*)(h + align_up(sizeof(int) * n_inst));
    double* hres = (double*)(h + 2 * align_up(sizeof(int) * n_inst));
    double* hbal = (double*)(h + 2 * align_up(sizeof(int) * n_inst) +
                             align_up(sizeof(double) * n_inst));
    if (!c->hip_ok(hipMemcpyAsync(hit, su.st.iter, sizeof(int) * n_inst,
                                  hipMemcpyDeviceToHost, c->stream), "copy") ||
        !c->hip_ok(hipMemcpyAsync(hst, su.st.status, sizeof(int) * n_inst,
                                  hipMemcpyDeviceToHost, c->stream), "copy") ||
        !c->hip_ok(hipMemcpyAsync(hres, su.st.resid, sizeof(double) * n_inst,
                                  hipMemcpyDeviceToHost, c->stream), "copy") ||
        !c->hip_ok(hipMemcpyAsync(hbal, su.d_bal, sizeof(double) * 3 * n_inst,
                                  hipMemcpyDeviceToHost, c->stream), "copy") ||
        !c->hip_ok(hipStreamSynchronize(c->stream), "sync"))
        return TR_ERR_HIP;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    tr_status worst = TR_OK;
    for (int i = 0; i < n_inst; ++i) {
        tr_status s = hst[i] == 0 ? TR_OK
                                  : (hst[i] == -4 ? TR_ERR_NONFINITE : TR_NOT_CONVERGED);
        if (s == TR_ERR_NONFINITE) c->fail("problem %d: non-finite iterate", i);
        if (stats) {
            stats[i].status = s;
            stats[i].iterations = hit[i];
            stats[i].residual = hres[i];
            const double sq = hbal[3 * i], sa = hbal[3 * i + 1], lk = hbal[3 * i + 2];
            stats[i].balance_rel = sq != 0.0 ? std::fabs(sq - sa - lk) / std::fabs(sq)
                                             : std::fabs(sa + lk);
            stats[i].seconds = secs;
        }
        if (s < 0 && (worst >= 0 || s < worst)) worst = s;
        else if (worst >= 0 && s > worst) worst = s;
    }
    c->last_sweeps = done_iters;
    return worst;
}

extern "C" tr_status tr_check_args(int32_t n_inst, const tr_problem* p,
                                   const tr_quadrature* q, double tol,
                                   int32_t max_iter, char* msg, int32_t msg_len) {
    Ctx c;
    tr_status s = TR_OK;
    DirTable* dt = new DirTable();
    if (!check_problems(&c, n_inst, p, true)) s = TR_ERR_INVALID_ARG;
    else if (!build_dirtable(&c, q, p[0].dim, dt)) s = TR_ERR_INVALID_ARG;
    else if (max_iter <= 0 || !std::isfinite(tol) || tol == 0.0) {
        c.fail("need max_iter > 0 and a finite non-zero tol");
        s = TR_ERR_INVALID_ARG;
    }
    delete dt;
    if (msg && msg_len > 0) {
        std::snprintf(msg, (size_t)msg_len, "%s", c.err.c_str());
    }
    return s;
}

// Tuning knobs for the autotuner and tests: force directions per lane (D),
// waves per workgroup (W), slices (S) and rows per segment (R); 0 = auto.
extern "C" tr_status tr_set_sweep_config(tr_context* ctx, int32_t D, int32_t W,
                                         int32_t S, int32_t R) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    const int okD[] = {0, 1, 2, 3, 4, 6, 9};
    bool good = false;
    for (int v : okD) good |= D == v;
    if (!good || W < 0 || W > 16 || S < 0 || R < 0 || R > 64 || (R & (R - 1))) {
        c->fail("sweep config out of range");
        return TR_ERR_INVALID_ARG;
    }
    c->force_D = D;
    c->force_W = W;
    c->force_S = S;
    c->force_R = R;
    return TR_OK;
}

// Measured launch-shape choice: every candidate (D, W) plan is timed with
// HIP events over `reps` sweeps of the caller's problems (emission = source),
// after one untimed sweep; the fastest stays forced on the context.
extern "C" tr_status tr_autotune(tr_context* ctx, int32_t n_inst, const tr_problem* p,
                                 const tr_quadrature* q, int32_t reps, int32_t* out6,
                                 double* best_ms) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!check_problems(c, n_inst, p, true)) return TR_ERR_INVALID_ARG;
    if (reps < 1 || reps > 100) {
        c->fail("reps must be in 1..100");
        return TR_ERR_INVALID_ARG;
    }
    size_t total = 0;
    std::vector<size_t> off(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        off[i] = total;
        total += align_up(sizeof(float) * (size_t)p[i].nx * (p[i].dim == 1 ? 1 : p[i].ny));
    }
    char* buf = nullptr;
    if (!c->hip_ok(hipMalloc(&buf, total), "hipMalloc")) return TR_ERR_OOM;
    std::vector<float*> outs(n_inst);
    std::vector<const float*> em(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        outs[i] = (float*)(buf + off[i]);
        em[i] = p[i].source;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    tr_status rc = TR_OK;
    const int sD = c->force_D, sW = c->force_W, sS = c->force_S, sR = c->force_R;
    int bestD = 0, bestW = 0;
    double best = 1e300;
    std::vector<std::array<int, 5>> seen;
    if (!c->hip_ok(hipEventCreate(&e0), "event") || !c->hip_ok(hipEventCreate(&e1), "event")) {
        rc = TR_ERR_HIP;
    } else if (p[0].dim == 2) {
        // time one (D, W) shape: one untimed sweep, then `nrep` timed ones,
        // each with the sum of its partial planes (their number depends on
        // the shape, and the iteration's combine reads them all); returns
        // ms per sweep, -1 if the shape is not feasible, -2 on a HIP error
        auto time_shape = [&](int D, int W, int nrep, std::array<int, 5>* key) -> double {
            c->force_D = D;
            c->force_W = W;
            c->force_S = 0;
            c->force_R = sR;
            Setup su;
            if (!c->setup(n_inst, p, q, nullptr, outs.data(), em.data(), &su)) {
                c->err.clear();
                return -1.0;   // shape not feasible (LDS)
            }
            if (key)
                *key = {su.plan.D, su.plan.W, su.plan.S[0], su.plan.KB, su.plan.fast ? 1 : 0};
            auto sweep = [&]() {
                if (!c->launch_sweep(su, n_inst, nullptr, nullptr, 0)) return false;
                launch_combine((int)su.blocks.size(), su.d_inst, su.d_blocks, nullptr,
                               su.d_red, 1, 0, c->stream, su.d_dt);
                return c->hip_ok(hipGetLastError(), "combine launch");
            };
            if (!sweep()) return -2.0;
            (void)hipEventRecord(e0, c->stream);
            for (int r = 0; r < nrep; ++r)
                if (!sweep()) return -2.0;
            (void)hipEventRecord(e1, c->stream);
            if (!c->hip_ok(hipEventSynchronize(e1), "sync")) return -2.0;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            return (double)ms / nrep;
        };
        struct Cand { int D, W; double ms; };
        std::vector<Cand> cands;
        const int Ds[] = {1, 2, 3, 4};
        // wave counts: a fixed set, and for one direction per lane every
        // W = ceil(nd/S) (the octant's nd directions in S full slices)
        std::vector<int> Ws = {0, 4, 6, 8, 9, 10, 12, 16};
        {
            DirTable dt1;
            if (build_dirtable(c, q, 2, &dt1)) {
                const int nd = dt1.count[0];
                for (int S = 1; S <= nd; ++S) {
                    const int w = (nd + S - 1) / S;
                    if (w >= 2 && std::find(Ws.begin(), Ws.end(), w) == Ws.end()) Ws.push_back(w);
                }
            }
            c->err.clear();
        }
        for (int D : Ds) {
            for (int W : Ws) {
                if (W != 0 && D > 1 && std::find(Ws.begin(), Ws.begin() + 8, W) == Ws.begin() + 8)
                    continue;   // the added counts are for D = 1
                if (W > sweep2d_max_w(D)) continue;
                std::array<int, 5> key{};
                // feasibility and the resolved shape first (no launch)
                {
                    c->force_D = D;
                    c->force_W = W;
                    c->force_S = 0;
                    c->force_R = sR;
                    Setup su;
                    if (!c->setup(n_inst, p, q, nullptr, outs.data(), em.data(), &su)) {
                        c->err.clear();
                        continue;
                    }
                    key = {su.plan.D, su.plan.W, su.plan.S[0], su.plan.KB, su.plan.fast ? 1 : 0};
                }
                if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
                seen.push_back(key);
                const double ms = time_shape(D, W, reps, nullptr);
                if (ms == -2.0) { rc = TR_ERR_HIP; break; }
                if (ms < 0.0) continue;
                cands.push_back({key[0], key[1], ms});
                if (ms < best) best = ms;
            }
            if (rc != TR_OK) break;
        }
        // the shapes within 5 % of the fastest are timed again in three
        // interleaved rounds (the first pass times each shape once, in a
        // fixed order, so clock changes and noise can bias it)
        std::vector<Cand> fin;
        for (const Cand& k : cands)
            if (k.ms <= 1.05 * best) fin.push_back({k.D, k.W, 0.0});
        if (fin.size() > 4) {
            std::sort(fin.begin(), fin.end(), [&](const Cand& x, const Cand& y) {
                auto msof = [&](const Cand& z) {
                    for (const Cand& k : cands)
                        if (k.D == z.D && k.W == z.W) return k.ms;
                    return 1e300;
                };
                return msof(x) < msof(y);
            });
            fin.resize(4);
        }
        const int rounds = fin.size() > 1 ? 3 : 0;
        for (int r = 0; r < rounds && rc == TR_OK; ++r)
            for (size_t k = 0; k < fin.size(); ++k) {
                Cand& f = fin[(k + (size_t)r) % fin.size()];
                const double ms = time_shape(f.D, f.W, reps, nullptr);
                if (ms < 0.0) { rc = TR_ERR_HIP; break; }
                f.ms += ms;
            }
        if (rc == TR_OK) {
            if (rounds > 0) {
                best = 1e300;
                for (const Cand& f : fin)
                    if (f.ms / rounds < best) {
                        best = f.ms / rounds;
                        bestD = f.D;
                        bestW = f.W;
                    }
            } else {
                for (const Cand& k : cands)
                    if (k.ms <= best) { bestD = k.D; bestW = k.W; }
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(buf);
    if (rc != TR_OK) {
        c->force_D = sD; c->force_W = sW; c->force_S = sS; c->force_R = sR;
        return rc;
    }
    if (bestD > 0) {
        c->force_D = bestD;
        c->force_W = bestW;
        c->force_S = 0;
    }
    if (best_ms) *best_ms = best < 1e299 ? best : 0.0;
    return out6 ? tr_get_sweep_plan(ctx, n_inst, p, q, out6) : TR_OK;
}

extern "C" tr_status tr_set_sweep_kernel(tr_context* ctx, int32_t generic) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    if (generic != 0 && generic != 1) {
        c->fail("generic must be 0 or 1");
        return TR_ERR_INVALID_ARG;
    }
    c->force_generic = generic != 0;
    return TR_OK;
}

extern "C" tr_status tr_set_persistent(tr_context* ctx, int32_t enable, int32_t spin_limit) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    if (enable != 0 && enable != 1) {
        c->fail("enable must be 0 or 1");
        return TR_ERR_INVALID_ARG;
    }
    c->persistent = enable != 0;
    c->persist_spin = spin_limit > 0 ? spin_limit : (1 << 18);
    return TR_OK;
}

extern "C" tr_status tr_profile_read_ex(tr_context* ctx, double* out6) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c || !out6) return TR_ERR_INVALID_ARG;
    for (int k = 0; k < 3; ++k) {
        out6[2 * k] = c->prof_ms[k];
        out6[2 * k + 1] = (double)c->prof_n[k];
    }
    return TR_OK;
}

extern "C" tr_status tr_set_sync_checks(tr_context* ctx, int32_t enable) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    if (enable != 0 && enable != 1) {
        c->fail("enable must be 0 or 1");
        return TR_ERR_INVALID_ARG;
    }
    c->sync_checks = enable != 0;
    return TR_OK;
}

extern "C" tr_status tr_set_stop_rule(tr_context* ctx, int32_t rule) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    if (rule != TR_STOP_CHANGE && rule != TR_STOP_ERROR_BOUND) {
        c->fail("unknown stopping rule %d", rule);
        return TR_ERR_INVALID_ARG;
    }
    c->stop_rule = rule;
    return TR_OK;
}

// Sweep launch plan the next call would use (for logs and the tuner).
extern "C" tr_status tr_get_sweep_plan(tr_context* ctx, int32_t n_inst,
                                       const tr_problem* p, const tr_quadrature* q,
                                       int32_t* out6) {
    Ctx tmp;
    Ctx* c = ctx ? reinterpret_cast<Ctx*>(ctx) : &tmp;
    if (!out6) return TR_ERR_INVALID_ARG;
    if (!check_problems(c, n_inst, p, false)) return TR_ERR_INVALID_ARG;
    DirTable* dt = new DirTable();
    if (!build_dirtable(c, q, p[0].dim, dt)) {
        delete dt;
        return TR_ERR_INVALID_ARG;
    }
    bool p1 = false;
    for (int i = 0; i < n_inst; ++i) p1 = p1 || p[i].sigma_s1 != nullptr;
    Plan pl = make_plan(c, n_inst, p, *dt, p1);
    delete dt;
    out6[0] = pl.D;
    out6[1] = pl.W;
    out6[2] = pl.S.empty() ? 0 : pl.S[0];
    out6[3] = pl.R.empty() ? 0 : pl.R[0];
    out6[4] = pl.KB;
    out6[5] = p[0].dim == 2 && pl.fast ? 1 : 0;
    return TR_OK;
}

// Kernel timing: enable != 0 starts (and resets) event timing of the sweep
// launches and of the combine+finalize pair inside tr_solve.
extern "C" tr_status tr_profile_enable(tr_context* ctx, int32_t enable) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->prof = enable != 0;
    c->ev_used = 0;
    for (int k = 0; k < 4; ++k) { c->prof_ms[k] = 0.0; c->prof_n[k] = 0; }
    return TR_OK;
}

extern "C" tr_status tr_profile_read(tr_context* ctx, double* out4) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c || !out4) return TR_ERR_INVALID_ARG;
    out4[0] = c->prof_ms[0];
    out4[1] = (double)c->prof_n[0];
    out4[2] = c->prof_ms[1];
    out4[3] = (double)c->prof_n[1];
    return TR_OK;
}
