// eigen_host.cpp -- tr_eigen: the one-group k-eigenvalue power iteration
// (section 5.2 Eq. 26; Appendix A2 Eq. A1-A4).  Each outer iteration runs
// the batched source iteration to tol_inner with the fission emission as
// source, warm-started from the current eigenfunction (the inner loop M),
// then the outer update P on the device (eigen.hip).  Instances finish
// independently: a finished instance keeps its last inner solution and is
// passed by the later inner solves.
#include <chrono>
#include <cmath>
#include <algorithm>
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
    if (!(tol_k > 0.0) || !(tol_phi > 0.0) || !std::isfinite(tol_k) ||
        !std::isfinite(tol_phi) || !std::isfinite(tol_inner) || tol_inner == 0.0 ||
        max_outer <= 0 || max_inner <= 0) {
        c->fail("need finite tol_k, tol_phi > 0, a finite non-zero tol_inner, "
                "max_outer > 0 and max_inner > 0");
        return TR_ERR_INVALID_ARG;
    }
    for (int i = 0; i < n_inst; ++i) {
        if (!nu_sigma_f[i] || !phi_out[i]) {
            c->fail("problem %d: null nu_sigma_f or phi_out", i);
            return TR_ERR_INVALID_ARG;
        }
        if (k_init && (!(k_init[i] > 0.0) || !std::isfinite(k_init[i]))) {
            c->fail("problem %d: k_init must be positive and finite", i);
            return TR_ERR_INVALID_ARG;
        }
    }
    // the problems as the inner solve sees them: the source is the fission
    // emission buffer (the caller's source field is not read)
    std::vector<tr_problem> pp(p, p + n_inst);
    for (int i = 0; i < n_inst; ++i) pp[i].source = pp[i].sigma_t;   // placeholder for the check
    if (!check_problems(c, n_inst, pp.data(), true)) return TR_ERR_INVALID_ARG;

    // eigen workspace: S and prev per instance, then the tables
    size_t off = 0;
    std::vector<size_t> offS(n_inst), offV(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const size_t cells = (size_t)pp[i].nx * (pp[i].dim == 1 ? 1 : pp[i].ny);
        offS[i] = off;
        off += align_up(sizeof(float) * cells);
        offV[i] = off;
        off += align_up(sizeof(float) * cells);
    }
    const size_t oSbytes = off;
    const size_t oDesc = off;
    off += align_up(sizeof(EigDesc) * n_inst);
    const size_t oState = off;
    off += align_up(sizeof(EigState) * n_inst);
    const size_t oDone = off;
    off += align_up(sizeof(int) * n_inst);
    if (!c->eig.reserve(c, off)) return TR_ERR_OOM;
    char* eb = (char*)c->eig.base;
    for (int i = 0; i < n_inst; ++i) pp[i].source = (const float*)(eb + offS[i]);
    EigDesc* d_desc = (EigDesc*)(eb + oDesc);
    EigState* d_state = (EigState*)(eb + oState);
    int* d_done = (int*)(eb + oDone);

    Setup su;
    if (!c->setup(n_inst, pp.data(), q, phi_out, phi_out, nullptr, &su))
        return c->err.rfind("out of", 0) == 0 ? TR_ERR_OOM : TR_ERR_INVALID_ARG;
    const size_t htab = off - oDesc;
    const size_t hread = align_up(sizeof(EigState) * n_inst) + align_up(sizeof(double) * 3 * n_inst) +
                         align_up(sizeof(int) * n_inst);
    // the setup's table upload reads the pinned buffer: wait for it first
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "sync")) return TR_ERR_HIP;
    if (!c->pinned.reserve(c, std::max(htab, hread) + align_up(sizeof(int) * n_inst)))
        return TR_ERR_OOM;
    char* h = (char*)c->pinned.ptr;
    std::memset(h, 0, htab);
    EigDesc* hd = (EigDesc*)h;
    EigState* hs = (EigState*)(h + (oState - oDesc));
    for (int i = 0; i < n_inst; ++i) {
        hd[i].nsf = nu_sigma_f[i];
        hd[i].phi0 = phi_init ? phi_init[i] : nullptr;
        hd[i].S = (float*)(eb + offS[i]);
        hd[i].prev = (float*)(eb + offV[i]);
        hd[i].vol = su.inst[i].dx * su.inst[i].dy;
        hs[i].k = k_init ? k_init[i] : 1.0;
        hs[i].status = 1;
    }
    if (!c->hip_ok(hipMemcpyAsync(eb + oDesc, h, htab, hipMemcpyHostToDevice, c->stream),
                   "table upload") ||
        !c->hip_ok(hipMemsetAsync(eb, 0, oSbytes, c->stream), "workspace clear"))
        return TR_ERR_HIP;
    const int nblocks = (int)su.blocks.size();
    launch_eig_start(n_inst, nblocks, su.d_inst, su.d_blocks, d_desc, d_state, d_done,
                     su.d_bpart, c->stream);
    if (!c->hip_ok(hipGetLastError(), "eigen start launch")) return TR_ERR_HIP;
    // cross sections and the first fission source, then the start's verdict
    tr_status s0 = c->scan_fields(su, n_inst, pp.data(), true, nullptr);
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
    for (int outer = 1; outer <= max_outer; ++outer) {
        launch_init(n_inst, nblocks, su.d_inst, su.d_blocks, su.d_dt, su.st, d_done, c->stream);
        if (!c->hip_ok(hipGetLastError(), "init launch")) return TR_ERR_HIP;
        int sw = 0;
        if (!c->si_iterate(su, n_inst, atol, norm_kind, max_inner, &sw)) return TR_ERR_HIP;
        total_sweeps += sw;
        launch_eig_update(n_inst, nblocks, su.d_inst, su.d_blocks, d_desc, d_state, d_done,
                          su.d_bpart, su.st, tol_k, tol_phi, outer == max_outer ? 1 : 0,
                          c->stream);
        if (!c->hip_ok(hipGetLastError(), "eigen update launch")) return TR_ERR_HIP;
        int* hdone = (int*)c->pinned.ptr;
        if (!c->hip_ok(hipMemcpyAsync(hdone, d_done, sizeof(int) * n_inst,
                                      hipMemcpyDeviceToHost, c->stream), "flag copy") ||
            !c->hip_ok(hipStreamSynchronize(c->stream), "sync"))
            return TR_ERR_HIP;
        bool all = true;
        for (int i = 0; i < n_inst; ++i) all &= hdone[i] != 0;
        if (all) break;
    }
    // balance of every instance's last inner solve, then its normalisation
    if (!c->si_balance(su, n_inst)) return TR_ERR_HIP;
    launch_eig_final(nblocks, su.d_inst, su.d_blocks, d_state, c->stream);
    if (!c->hip_ok(hipGetLastError(), "eigen final launch")) return TR_ERR_HIP;
    EigState* rs = (EigState*)h;
    double* rb = (double*)(h + align_up(sizeof(EigState) * n_inst));
    if (!c->hip_ok(hipMemcpyAsync(rs, d_state, sizeof(EigState) * n_inst,
                                  hipMemcpyDeviceToHost, c->stream), "copy") ||
        !c->hip_ok(hipMemcpyAsync(rb, su.d_bal, sizeof(double) * 3 * n_inst,
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
            const double sq = rb[3 * i], sa = rb[3 * i + 1], lk = rb[3 * i + 2];
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
