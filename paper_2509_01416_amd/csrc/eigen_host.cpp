// eigen_host.cpp -- tr_eigen and tr_eigen_mg: k-eigenvalue power iteration
// (one group: section 5.2 Eq. 26; G groups with downscatter: section 5.3
// Eq. 27-29; the loop of Appendix A2 Eq. A1-A4).  Each outer iteration runs
// the batched source iteration to tol_inner as the inner loop M, warm-started
// from the current eigenfunction: with one group its source is the fission
// emission; with G groups the groups are solved in order (Gauss-Seidel in
// energy), each with chi_g times the previous iterate's fission density plus
// the downscatter of the groups already solved.  Then the outer update P on
// the device (eigen.hip).  Problems finish independently: a finished problem
// keeps its last inner solution and is passed by the later inner solves.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "mdpnop.h"
#include "eigen_kernels.h"
#include "host_internal.h"

namespace mdp {
void launch_init(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                 const DirTable* dt, IterState st, const int* skip, hipStream_t s);
}

using namespace mdp;

namespace {

// One call's problems as the inner solve sees them: N = n_inst * G
// pseudo-problems j = g*n_inst + i, group-major so that one group's sweep
// workgroups are contiguous in launch order (the source pointers are filled
// in here).
struct EigCall {
    int n_inst = 0, G = 1;
    std::vector<tr_problem> pp;                 // N
    std::vector<const float*> nsf;              // N
    std::vector<const float*> phi0;             // N (nullptr entries: flat start)
    std::vector<float*> phi;                    // N
    std::vector<double> k0;                     // n_inst
    std::vector<float> chi;                     // n_inst * G (multigroup)
    std::vector<const float*> down;             // n_inst * kMaxGroups^2 (h -> g, h < g)
};

tr_status run_eigen(Ctx* c, EigCall& e, const tr_quadrature* q, double tol_k, double tol_phi,
                    double tol_inner, int max_outer, int max_inner, tr_eigen_stats* stats,
                    std::chrono::steady_clock::time_point t0) {
    const int n_inst = e.n_inst, G = e.G, N = n_inst * G;
    // workspace: S and prev per pseudo-problem, fd per problem (G > 1), tables
    size_t off = 0;
    std::vector<size_t> offS(N), offV(N), offF(n_inst);
    for (int j = 0; j < N; ++j) {
        const size_t cells = (size_t)e.pp[j].nx * (e.pp[j].dim == 1 ? 1 : e.pp[j].ny);
        offS[j] = off;
        off += align_up(sizeof(float) * cells);
        offV[j] = off;
        off += align_up(sizeof(float) * cells);
    }
    if (G > 1)
        for (int i = 0; i < n_inst; ++i) {
            const tr_problem& P = e.pp[i];
            const size_t cells = (size_t)P.nx * (P.dim == 1 ? 1 : P.ny);
            offF[i] = off;
            off += align_up(sizeof(float) * cells);
        }
    const size_t oSbytes = off;
    const size_t oDesc = off;
    off += align_up(sizeof(EigDesc) * N);
    const size_t oState = off;
    off += align_up(sizeof(EigState) * n_inst);
    const size_t oDone = off;
    off += align_up(sizeof(int) * n_inst);
    const size_t oMg = off;
    off += G > 1 ? align_up(sizeof(MgDesc) * n_inst) : 0;
    const size_t oSkip = off;
    off += G > 1 ? align_up(sizeof(int) * N) : 0;
    if (!c->eig.reserve(c, off)) return TR_ERR_OOM;
    char* eb = (char*)c->eig.base;
    for (int j = 0; j < N; ++j) e.pp[j].source = (const float*)(eb + offS[j]);
    EigDesc* d_desc = (EigDesc*)(eb + oDesc);
    EigState* d_state = (EigState*)(eb + oState);
    int* d_done = (int*)(eb + oDone);
    MgDesc* d_mg = G > 1 ? (MgDesc*)(eb + oMg) : nullptr;
    int* d_skip = G > 1 ? (int*)(eb + oSkip) : d_done;

    // A multigroup inner solve sweeps one group's n_inst problems at a time:
    // unless the caller forced a launch shape, plan it for those (group 0's
    // problems, the first n_inst in group-major order) rather than for all
    // N, whose plan would leave a group pass short of workgroups.
    const int saved_D = c->force_D, saved_W = c->force_W, saved_S = c->force_S;
    const bool replan = G > 1 && e.pp[0].dim == 2 && c->force_W <= 0;
    if (replan) {
        DirTable dt;
        if (!build_dirtable(c, q, 2, &dt)) return TR_ERR_INVALID_ARG;
        const Plan pl = make_plan(c, n_inst, e.pp.data(), dt);
        int smin = pl.S[0];
        for (int v : pl.S) smin = std::min(smin, v);
        c->force_D = pl.D;
        c->force_W = pl.W;
        c->force_S = smin;
    }
    Setup su;
    const bool set_ok = c->setup(N, e.pp.data(), q, e.phi.data(), e.phi.data(), nullptr, &su);
    if (replan) {
        c->force_D = saved_D;
        c->force_W = saved_W;
        c->force_S = saved_S;
    }
    if (!set_ok)
        return c->err.rfind("out of", 0) == 0 ? TR_ERR_OOM : TR_ERR_INVALID_ARG;
    const size_t htab = oSkip - oDesc;
    const size_t hread = align_up(sizeof(EigState) * n_inst) + align_up(sizeof(double) * 3 * N);
    // the setup's table upload reads the pinned buffer: wait for it first
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "sync")) return TR_ERR_HIP;
    if (!c->pinned.reserve(c, std::max(htab, hread) + 2 * align_up(sizeof(int) * N)))
        return TR_ERR_OOM;
    char* h = (char*)c->pinned.ptr;
    std::memset(h, 0, htab);
    EigDesc* hd = (EigDesc*)h;
    EigState* hs = (EigState*)(h + (oState - oDesc));
    MgDesc* hm = (MgDesc*)(h + (oMg - oDesc));
    for (int j = 0; j < N; ++j) {
        hd[j].nsf = e.nsf[j];
        hd[j].phi0 = e.phi0[j];
        hd[j].S = (float*)(eb + offS[j]);
        hd[j].prev = (float*)(eb + offV[j]);
        hd[j].vol = su.inst[j].dx * su.inst[j].dy;
    }
    for (int i = 0; i < n_inst; ++i) {
        hs[i].k = e.k0[i];
        hs[i].status = 1;
        if (G > 1) {
            hm[i].fd = (float*)(eb + offF[i]);
            for (int g = 0; g < G; ++g) hm[i].chi[g] = e.chi[(size_t)i * G + g];
            for (int t = 0; t < kMaxGroups * kMaxGroups; ++t)
                hm[i].ss[t] = e.down[(size_t)i * kMaxGroups * kMaxGroups + t];
        }
    }
    if (!c->hip_ok(hipMemcpyAsync(eb + oDesc, h, htab, hipMemcpyHostToDevice, c->stream),
                   "table upload") ||
        !c->hip_ok(hipMemsetAsync(eb, 0, oSbytes, c->stream), "workspace clear"))
        return TR_ERR_HIP;
    const int nblocks = (int)su.blocks.size();
    launch_eig_start(n_inst, G, nblocks, su.d_inst, su.d_blocks, d_desc, d_state, d_done,
                     su.d_bpart, c->stream);
    if (!c->hip_ok(hipGetLastError(), "eigen start launch")) return TR_ERR_HIP;
    // cross sections and the first sources, then the start's verdict
    tr_status s0 = c->scan_fields(su, N, e.pp.data(), true, nullptr);
    if (s0 < 0) return s0;
    if (!c->hip_ok(hipMemcpyAsync(h, d_state, sizeof(EigState) * n_inst, hipMemcpyDeviceToHost,
                                  c->stream), "state copy") ||
        !c->hip_ok(hipStreamSynchronize(c->stream), "sync"))
        return TR_ERR_HIP;
    for (int i = 0; i < n_inst; ++i)
        if (((EigState*)h)[i].status < 0) {
            c->fail("problem %d: nu_sigma_f must be finite and >= 0 and the starting "
                    "flux finite with F(phi) > 0", i);
            return TR_ERR_INVALID_ARG;
        }

    const int norm_kind = tol_inner < 0 ? 1 : 0;
    const double atol = std::fabs(tol_inner);
    int total_sweeps = 0;
    // a warm inner solve usually needs about as many sweeps as the previous
    // one of its group: its first chunk takes that many (the most any running
    // problem needed) before the first read-back of the done flags
    std::vector<int> last_sw(G, 4), running(n_inst, 1);
    int* hiters = (int*)((char*)c->pinned.ptr + align_up(sizeof(int) * N));
    for (int outer = 1; outer <= max_outer; ++outer) {
        if (G > 1) launch_mg_fission(n_inst, G, nblocks, su.d_inst, su.d_blocks, d_desc, d_mg, d_state,
                                     d_done, c->stream);
        for (int g = 0; g < G; ++g) {
            if (G > 1) launch_mg_group(N, G, g, nblocks, su.d_inst, su.d_blocks, d_desc, d_mg,
                                       d_done, d_skip, c->stream);
            launch_init(N, nblocks, su.d_inst, su.d_blocks, su.d_dt, su.st, d_skip, c->stream);
            if (!c->hip_ok(hipGetLastError(), "init launch")) return TR_ERR_HIP;
            int sw = 0;
            if (!c->si_iterate(su, N, atol, norm_kind, max_inner, &sw, last_sw[g], hiters))
                return TR_ERR_HIP;
            total_sweeps += sw;
            int need = 1;
            for (int i = 0; i < n_inst; ++i)
                if (running[i]) need = std::max(need, hiters[g * n_inst + i]);
            last_sw[g] = need;
        }
        launch_eig_update(n_inst, G, nblocks, su.d_inst, su.d_blocks, d_desc, d_state, d_done,
                          su.d_bpart, su.st, tol_k, tol_phi, outer == max_outer ? 1 : 0,
                          c->stream);
        if (!c->hip_ok(hipGetLastError(), "eigen update launch")) return TR_ERR_HIP;
        int* hdone = (int*)c->pinned.ptr;
        if (!c->hip_ok(hipMemcpyAsync(hdone, d_done, sizeof(int) * n_inst,
                                      hipMemcpyDeviceToHost, c->stream), "flag copy") ||
            !c->hip_ok(hipStreamSynchronize(c->stream), "sync"))
            return TR_ERR_HIP;
        bool all = true;
        for (int i = 0; i < n_inst; ++i) {
            running[i] = hdone[i] == 0;
            all &= hdone[i] != 0;
        }
        if (all) break;
    }
    // balance of every problem's last inner solve, then its normalisation
    if (!c->si_balance(su, N)) return TR_ERR_HIP;
    launch_eig_final(n_inst, nblocks, su.d_inst, su.d_blocks, d_state, c->stream);
    if (!c->hip_ok(hipGetLastError(), "eigen final launch")) return TR_ERR_HIP;
    EigState* rs = (EigState*)h;
    double* rb = (double*)(h + align_up(sizeof(EigState) * n_inst));
    if (!c->hip_ok(hipMemcpyAsync(rs, d_state, sizeof(EigState) * n_inst,
                                  hipMemcpyDeviceToHost, c->stream), "copy") ||
        !c->hip_ok(hipMemcpyAsync(rb, su.d_bal, sizeof(double) * 3 * N,
                                  hipMemcpyDeviceToHost, c->stream), "copy") ||
        !c->hip_ok(hipStreamSynchronize(c->stream), "sync"))
        return TR_ERR_HIP;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    tr_status worst = TR_OK;
    for (int i = 0; i < n_inst; ++i) {
        const EigState& E = rs[i];
        const tr_status s = E.status == 0 ? TR_OK
                            : E.status == -4 ? TR_ERR_NONFINITE : TR_NOT_CONVERGED;
        if (s == TR_ERR_NONFINITE) c->fail("problem %d: non-finite iterate", i);
        if (stats) {
            tr_eigen_stats& o = stats[i];
            o.status = s;
            o.outer = E.outer;
            o.inner = E.inner;
            o.k = E.k;
            o.dk = E.dk;
            o.dphi = E.dphi;
            // the group balances summed (each group: its sources against its
            // removal and leakage)
            double sq = 0.0, sa = 0.0, lk = 0.0;
            for (int g = 0; g < G; ++g) {
                const size_t j = (size_t)g * n_inst + i;
                sq += rb[3 * j];
                sa += rb[3 * j + 1];
                lk += rb[3 * j + 2];
            }
            o.balance_rel = sq != 0.0 ? std::fabs(sq - sa - lk) / std::fabs(sq)
                                      : std::fabs(sa + lk);
            o.seconds = secs;
        }
        if (s < 0 && (worst >= 0 || s < worst)) worst = s;
        else if (worst >= 0 && s > worst) worst = s;
    }
    c->last_sweeps = total_sweeps;
    return worst;
}

bool check_tolerances(Ctx* c, double tol_k, double tol_phi, double tol_inner, int max_outer,
                      int max_inner) {
    if (!(tol_k > 0.0) || !(tol_phi > 0.0) || !std::isfinite(tol_k) ||
        !std::isfinite(tol_phi) || !std::isfinite(tol_inner) || tol_inner == 0.0 ||
        max_outer <= 0 || max_inner <= 0) {
        c->fail("need finite tol_k, tol_phi > 0, a finite non-zero tol_inner, "
                "max_outer > 0 and max_inner > 0");
        return false;
    }
    return true;
}

}  // namespace

extern "C" tr_status tr_eigen(tr_context* ctx, int32_t n_inst, const tr_problem* p,
                              const float* const* nu_sigma_f, const tr_quadrature* q,
                              const float* const* phi_init, float* const* phi_out,
                              const double* k_init, double tol_k, double tol_phi,
                              double tol_inner, int32_t max_outer, int32_t max_inner,
                              tr_eigen_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (n_inst <= 0 || !p || !nu_sigma_f || !phi_out) {
        c->fail("need n_inst > 0 problems, nu_sigma_f and phi_out");
        return TR_ERR_INVALID_ARG;
    }
    if (!check_tolerances(c, tol_k, tol_phi, tol_inner, max_outer, max_inner))
        return TR_ERR_INVALID_ARG;
    EigCall e;
    e.n_inst = n_inst;
    e.G = 1;
    e.pp.assign(p, p + n_inst);
    for (int i = 0; i < n_inst; ++i) {
        if (!nu_sigma_f[i] || !phi_out[i]) {
            c->fail("problem %d: null nu_sigma_f or phi_out", i);
            return TR_ERR_INVALID_ARG;
        }
        if (k_init && (!(k_init[i] > 0.0) || !std::isfinite(k_init[i]))) {
            c->fail("problem %d: k_init must be positive and finite", i);
            return TR_ERR_INVALID_ARG;
        }
        e.pp[i].source = e.pp[i].sigma_t;   // placeholder for the check
        e.nsf.push_back(nu_sigma_f[i]);
        e.phi0.push_back(phi_init ? phi_init[i] : nullptr);
        e.phi.push_back(phi_out[i]);
        e.k0.push_back(k_init ? k_init[i] : 1.0);
    }
    if (!check_problems(c, n_inst, e.pp.data(), true) ||
        reject_anisotropic(c, n_inst, e.pp.data(), "tr_eigen"))
        return TR_ERR_INVALID_ARG;
    return run_eigen(c, e, q, tol_k, tol_phi, tol_inner, max_outer, max_inner, stats, t0);
}

extern "C" tr_status tr_eigen_mg(tr_context* ctx, int32_t n_inst, const tr_problem* geom,
                                 const tr_multigroup* mg, const tr_quadrature* q,
                                 const float* const* phi_init, float* const* phi_out,
                                 const double* k_init, double tol_k, double tol_phi,
                                 double tol_inner, int32_t max_outer, int32_t max_inner,
                                 tr_eigen_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (n_inst <= 0 || !geom || !mg || !phi_out) {
        c->fail("need n_inst > 0 problems, multigroup data and phi_out");
        return TR_ERR_INVALID_ARG;
    }
    if (!check_tolerances(c, tol_k, tol_phi, tol_inner, max_outer, max_inner))
        return TR_ERR_INVALID_ARG;
    const int G = mg[0].n_groups;
    if (G < 1 || G > kMaxGroups) {
        c->fail("n_groups must be 1..%d", kMaxGroups);
        return TR_ERR_INVALID_ARG;
    }
    EigCall e;
    e.n_inst = n_inst;
    e.G = G;
    const size_t N = (size_t)n_inst * G;
    e.pp.resize(N);
    e.nsf.resize(N);
    e.phi0.resize(N);
    e.phi.resize(N);
    e.chi.resize(N);
    e.down.assign((size_t)n_inst * kMaxGroups * kMaxGroups, nullptr);
    for (int i = 0; i < n_inst; ++i) {
        const tr_multigroup& m = mg[i];
        if (m.n_groups != G || !m.sigma_t || !m.sigma_s || !m.nu_sigma_f || !m.chi) {
            c->fail("problem %d: every problem needs the same n_groups and all tables", i);
            return TR_ERR_INVALID_ARG;
        }
        if (k_init && (!(k_init[i] > 0.0) || !std::isfinite(k_init[i]))) {
            c->fail("problem %d: k_init must be positive and finite", i);
            return TR_ERR_INVALID_ARG;
        }
        double chisum = 0.0;
        for (int g = 0; g < G; ++g) {
            const double x = m.chi[g];
            if (!(x >= 0.0) || !std::isfinite(x)) {
                c->fail("problem %d: chi[%d] must be finite and >= 0", i, g);
                return TR_ERR_INVALID_ARG;
            }
            chisum += x;
            for (int hh = 0; hh < g; ++hh)
                if (m.sigma_s[(size_t)g * G + hh]) {
                    c->fail("problem %d: upscatter %d -> %d is not supported", i, g, hh);
                    return TR_ERR_INVALID_ARG;
                }
            const size_t u = (size_t)i * G + g;           // caller's layout
            const size_t j = (size_t)g * n_inst + i;      // pseudo-problem
            if (!m.sigma_t[g] || !m.sigma_s[(size_t)g * G + g] || !m.nu_sigma_f[g] ||
                !phi_out[u]) {
                c->fail("problem %d group %d: need sigma_t, the within-group sigma_s, "
                        "nu_sigma_f and phi_out", i, g);
                return TR_ERR_INVALID_ARG;
            }
            tr_problem P = geom[i];
            P.sigma_t = m.sigma_t[g];
            P.sigma_s = m.sigma_s[(size_t)g * G + g];
            P.source = P.sigma_t;   // placeholder for the check
            e.pp[j] = P;
            e.nsf[j] = m.nu_sigma_f[g];
            e.phi0[j] = phi_init ? phi_init[u] : nullptr;
            e.phi[j] = phi_out[u];
            e.chi[u] = (float)x;
            for (int hh = g + 1; hh < G; ++hh)
                e.down[((size_t)i * kMaxGroups + g) * kMaxGroups + hh] =
                    m.sigma_s[(size_t)g * G + hh];
        }
        if (!(chisum > 0.0)) {
            c->fail("problem %d: chi must not vanish", i);
            return TR_ERR_INVALID_ARG;
        }
        e.k0.push_back(k_init ? k_init[i] : 1.0);
    }
    if (!check_problems(c, n_inst * G, e.pp.data(), true) ||
        reject_anisotropic(c, n_inst * G, e.pp.data(), "tr_eigen_mg"))
        return TR_ERR_INVALID_ARG;
    return run_eigen(c, e, q, tol_k, tol_phi, tol_inner, max_outer, max_inner, stats, t0);
}
