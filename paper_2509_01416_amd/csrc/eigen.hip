// eigen.hip -- outer update P of the one-group k-eigenvalue power iteration
// (section 5.2 Eq. 26; Appendix A2 Eq. A1-A4).  The inner solve M is the
// source iteration of si_kernels.hip / sweep2d.hip with the fission emission
// as its source.
//
// Update after an inner solve phi_half (per instance, FP64 sums):
//   F(phi)  = sum_cells nu_sigma_f * phi * V
//   k_new   = k * F(phi_half) / F(phi)
//   phi_new = phi_half / F(phi_half)                (normalisation F = 1)
//   S_new   = nu_sigma_f * phi_new / k_new           (next fission source)
// Converged when |k_new - k| / k_new < tol_k and
// max|phi_new - phi| / max|phi_new| < tol_phi.
//
// Multigroup problems (section 5.3, Eq. 27-29) run G groups of an instance
// as the pseudo-instances j = g*n_inst + i of the inner solve (group-major,
// so that one group's workgroups are contiguous in launch order); F sums over the
// groups and the change norm takes the maximum over them.  The inner source
// of group g is chi_g * fission density + downscatter (mg kernels below);
// with G = 1 it is the fission emission S written by the update.
//
// Per-block kernels take one reduction block (kCombineChunk cells of one
// pseudo-instance) per 256-thread workgroup and leave their partials in
// part[3 * slot ...]; per-instance kernels sum them in group and block
// order, so every result is independent of scheduling.
#include "eigen_kernels.h"

namespace mdp {

namespace {

constexpr int kThreads = 256;

// Deterministic in-block reductions of three values (fixed tree).
struct Red3 {
    double v[3][kThreads];
};

__device__ void reduce3(Red3& sh, double a, double b, double c, bool max_bc) {
    const int t = threadIdx.x;
    sh.v[0][t] = a;
    sh.v[1][t] = b;
    sh.v[2][t] = c;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (t < o) {
            sh.v[0][t] += sh.v[0][t + o];
            if (max_bc) {
                sh.v[1][t] = fmax(sh.v[1][t], sh.v[1][t + o]);
                sh.v[2][t] = fmax(sh.v[2][t], sh.v[2][t + o]);
            } else {
                sh.v[1][t] += sh.v[1][t + o];
                sh.v[2][t] += sh.v[2][t + o];
            }
        }
        __syncthreads();
    }
}

// The normalised value of a cell, computed identically wherever it is needed.
__device__ __forceinline__ float scaled(float phi, double sc) {
    return (float)((double)phi * sc);
}

__device__ __forceinline__ float fission(float nsf, float phi, double k) {
    return (float)((double)nsf * (double)phi / k);
}

// phi = phi0 or 1; partials: F(phi) / V and the count of invalid values.
__global__ void __launch_bounds__(kThreads)
eig_init_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                const EigDesc* __restrict__ ed, double* __restrict__ part) {
    __shared__ Red3 sh;
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0) return;
    const InstDesc& I = insts[bi.x];
    const EigDesc& E = ed[bi.x];
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    double s = 0.0, bad = 0.0;
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads) {
        const float p = E.phi0 != nullptr ? E.phi0[c] : 1.0f;
        const float f = E.nsf[c];
        I.phi[c] = p;
        if (!(f >= 0.f) || !isfinite(f) || !isfinite(p)) bad += 1.0;
        s += (double)f * (double)p;
    }
    reduce3(sh, s, bad, 0.0, false);
    if (threadIdx.x == 0) {
        part[3 * bi.z + 0] = sh.v[0][0];
        part[3 * bi.z + 1] = sh.v[1][0];
        part[3 * bi.z + 2] = 0.0;
    }
}

// First normalisation: rejects invalid data and a start without fissions.
__global__ void eig_init_fin_kernel(const InstDesc* __restrict__ insts,
                                    const EigDesc* __restrict__ ed, EigState* __restrict__ es,
                                    int* __restrict__ edone, const double* __restrict__ part,
                                    int n_inst, int G) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_inst) return;
    double F = 0.0, bad = 0.0;
    for (int g = 0; g < G; ++g) {
        const InstDesc& I = insts[g * n_inst + n];
        for (int b = 0; b < I.nred; ++b) {
            F += part[3 * (I.red0 + b)];
            bad += part[3 * (I.red0 + b) + 1];
        }
    }
    F *= ed[n].vol;
    if (bad > 0.0 || !isfinite(F) || !(F > 0.0) || !(es[n].k > 0.0)) {
        es[n].status = -1;
        edone[n] = 1;
        return;
    }
    es[n].scale = 1.0 / F;
}

// F(phi_half) / V partials of the inner solution.
__global__ void __launch_bounds__(kThreads)
eig_sum_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
               const EigDesc* __restrict__ ed, const int* __restrict__ edone,
               double* __restrict__ part, int NI) {
    __shared__ Red3 sh;
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || edone[bi.x % NI]) return;
    const InstDesc& I = insts[bi.x];
    const float* nsf = ed[bi.x].nsf;
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    double s = 0.0;
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads)
        s += (double)nsf[c] * (double)I.phi[c];
    reduce3(sh, s, 0.0, 0.0, false);
    if (threadIdx.x == 0) part[3 * bi.z] = sh.v[0][0];
}

// New eigenvalue and normalisation factor (one thread per instance).
__global__ void eig_k_kernel(const InstDesc* __restrict__ insts, const EigDesc* __restrict__ ed,
                             EigState* __restrict__ es, int* __restrict__ edone,
                             const double* __restrict__ part, IterState st, int n_inst, int G) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_inst || edone[n]) return;
    EigState& E = es[n];
    double F = 0.0;
    bool bad = false;
    for (int g = 0; g < G; ++g) {
        const InstDesc& I = insts[g * n_inst + n];
        for (int b = 0; b < I.nred; ++b) F += part[3 * (I.red0 + b)];
        bad |= st.status[g * n_inst + n] == -4;
    }
    F *= ed[n].vol;
    if (bad || !isfinite(F) || !(F > 0.0)) {
        E.status = -4;
        edone[n] = 1;
        return;
    }
    const double k_new = E.k * F / E.F;
    E.dk = fabs(k_new - E.k) / fabs(k_new);
    E.k = k_new;
    E.scale = 1.0 / F;
}

// Change partials of the normalised iterate against the previous one:
// F(phi_new) / V, max|phi_new - prev|, max|phi_new|.  mode 0 (start) writes
// the normalised iterate, the previous iterate and the fission source
// instead of comparing.
__global__ void __launch_bounds__(kThreads)
eig_diff_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                const EigDesc* __restrict__ ed, const EigState* __restrict__ es,
                const int* __restrict__ edone, double* __restrict__ part, int mode, int NI,
                int G) {
    __shared__ Red3 sh;
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || edone[bi.x % NI]) return;
    const InstDesc& I = insts[bi.x];
    const EigDesc& E = ed[bi.x];
    const double sc = es[bi.x % NI].scale, k = es[bi.x % NI].k;
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    double s = 0.0, d = 0.0, m = 0.0;
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads) {
        const float p = scaled(I.phi[c], sc);
        const float f = E.nsf[c];
        s += (double)f * (double)p;
        if (mode == 0) {
            I.phi[c] = p;
            E.prev[c] = p;
            if (G == 1) E.S[c] = fission(f, p, k);
        } else {
            d = fmax(d, fabs((double)p - (double)E.prev[c]));
            m = fmax(m, fabs((double)p));
        }
    }
    reduce3(sh, s, d, m, true);
    if (threadIdx.x == 0) {
        part[3 * bi.z + 0] = sh.v[0][0];
        part[3 * bi.z + 1] = sh.v[1][0];
        part[3 * bi.z + 2] = sh.v[2][0];
    }
}

// F of the stored iterate; after an inner solve (mode 1) also the change
// norm, the counters and the convergence decision.
__global__ void eig_conv_kernel(const InstDesc* __restrict__ insts,
                                const EigDesc* __restrict__ ed, EigState* __restrict__ es,
                                int* __restrict__ edone, const double* __restrict__ part,
                                IterState st, int n_inst, double tol_k, double tol_phi,
                                int mode, int last, int G) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_inst || edone[n]) return;
    EigState& E = es[n];
    double F = 0.0, d = 0.0, m = 0.0;
    for (int g = 0; g < G; ++g) {
        const InstDesc& I = insts[g * n_inst + n];
        for (int b = 0; b < I.nred; ++b) {
            const double* v = part + 3 * (size_t)(I.red0 + b);
            F += v[0];
            d = fmax(d, v[1]);
            m = fmax(m, v[2]);
        }
    }
    E.F = F * ed[n].vol;
    if (mode == 0) return;
    E.dphi = m > 0.0 ? d / m : INFINITY;
    E.outer += 1;
    for (int g = 0; g < G; ++g) E.inner += st.iter[g * n_inst + n];
    if (E.dk < tol_k && E.dphi < tol_phi) {
        E.status = 0;
        edone[n] = 1;
    } else if (last) {
        edone[n] = 1;
    }
}

// Next outer iterate of the running instances: phi_new, prev, S_new.
__global__ void __launch_bounds__(kThreads)
eig_apply_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                 const EigDesc* __restrict__ ed, const EigState* __restrict__ es,
                 const int* __restrict__ edone, int NI, int G) {
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || edone[bi.x % NI]) return;
    const InstDesc& I = insts[bi.x];
    const EigDesc& E = ed[bi.x];
    const double sc = es[bi.x % NI].scale, k = es[bi.x % NI].k;
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads) {
        const float p = scaled(I.phi[c], sc);
        I.phi[c] = p;
        E.prev[c] = p;
        if (G == 1) E.S[c] = fission(E.nsf[c], p, k);
    }
}

// Multigroup: fission density fd = sum_g nu_sigma_f_g phi_g / k of the
// stored iterate, one pass over the blocks of each instance's group 0 (all
// groups share the grid and the block layout).
__global__ void __launch_bounds__(kThreads)
mg_fission_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                  const EigDesc* __restrict__ ed, const MgDesc* __restrict__ md,
                  const EigState* __restrict__ es, const int* __restrict__ edone, int NI,
                  int G) {
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || bi.x >= NI || edone[bi.x]) return;   // the blocks of group 0
    const int n = bi.x;
    const double k = es[n].k;
    const int cells = insts[bi.x].cells;
    const int c1 = min(bi.y + kCombineChunk, cells);
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads) {
        double f = 0.0;
        for (int g = 0; g < G; ++g)
            f += (double)ed[g * NI + n].nsf[c] * (double)insts[g * NI + n].phi[c];
        md[n].fd[c] = (float)(f / k);
    }
}

// Multigroup: the source of group g, chi_g fd + sum_{h<g} sigma_s^{h->g}
// phi_h (the groups above g already hold this pass's solution), into the
// inner solve's source buffer S of pseudo-instance (n, g).
__global__ void __launch_bounds__(kThreads)
mg_source_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                 const EigDesc* __restrict__ ed, const MgDesc* __restrict__ md,
                 const int* __restrict__ edone, int NI, int g) {
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || bi.x / NI != g || edone[bi.x % NI]) return;
    const int n = bi.x % NI;
    const MgDesc& D = md[n];
    const float chi = D.chi[g];
    float* S = ed[bi.x].S;
    const int c1 = min(bi.y + kCombineChunk, insts[bi.x].cells);
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads) {
        double q = (double)chi * (double)D.fd[c];
        for (int h = 0; h < g; ++h) {
            const float* sd = D.ss[h * kMaxGroups + g];
            if (sd != nullptr) q += (double)sd[c] * (double)insts[h * NI + n].phi[c];
        }
        S[c] = (float)q;
    }
}

// Multigroup: pseudo-instances outside group g, or of finished instances,
// are skipped by the next inner solve.
__global__ void mg_mask_kernel(const int* __restrict__ edone, int* __restrict__ skip, int N,
                               int NI, int g) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    skip[j] = (j / NI != g || edone[j % NI]) ? 1 : 0;
}

// Emission of one source-iteration sweep from the current iterate u with
// the fission term taken from u: Q = sigma_s u + nu_sigma_f u / k.
__global__ void __launch_bounds__(kThreads)
eig_emission_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                    const EigDesc* __restrict__ ed, const EigState* __restrict__ es,
                    const int* __restrict__ edone) {   // one group (G = 1)
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || edone[bi.x]) return;
    const InstDesc& I = insts[bi.x];
    const EigDesc& E = ed[bi.x];
    const double k = es[bi.x].k;
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads) {
        const double u = I.phi[c];
        I.Q[c] = (float)((double)I.ss[c] * u + (double)E.nsf[c] * u / k);
    }
}

__global__ void __launch_bounds__(kThreads)
eig_final_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                 const EigState* __restrict__ es, int NI) {
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || es[bi.x % NI].status < 0) return;
    const InstDesc& I = insts[bi.x];
    const double sc = es[bi.x % NI].scale;
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    for (int c = bi.y + threadIdx.x; c < c1; c += kThreads) I.phi[c] = scaled(I.phi[c], sc);
}

}  // namespace

void launch_eig_start(int n_inst, int G, int nblocks, const InstDesc* insts, const int4* blocks,
                      const EigDesc* ed, EigState* es, int* edone, double* part,
                      hipStream_t s) {
    const dim3 gi((n_inst + 63) / 64), bi(64);
    hipLaunchKernelGGL(eig_init_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks,
                       ed, part);
    hipLaunchKernelGGL(eig_init_fin_kernel, gi, bi, 0, s, insts, ed, es, edone, part, n_inst, G);
    hipLaunchKernelGGL(eig_diff_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks, ed,
                       es, edone, part, 0, n_inst, G);
    hipLaunchKernelGGL(eig_conv_kernel, gi, bi, 0, s, insts, ed, es, edone, part, IterState{},
                       n_inst, 0.0, 0.0, 0, 0, G);
}

void launch_eig_update(int n_inst, int G, int nblocks, const InstDesc* insts, const int4* blocks,
                       const EigDesc* ed, EigState* es, int* edone, double* part,
                       IterState st, double tol_k, double tol_phi, int last, hipStream_t s) {
    const dim3 gi((n_inst + 63) / 64), bi(64);
    hipLaunchKernelGGL(eig_sum_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks, ed,
                       edone, part, n_inst);
    hipLaunchKernelGGL(eig_k_kernel, gi, bi, 0, s, insts, ed, es, edone, part, st, n_inst, G);
    hipLaunchKernelGGL(eig_diff_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks, ed,
                       es, edone, part, 1, n_inst, G);
    hipLaunchKernelGGL(eig_conv_kernel, gi, bi, 0, s, insts, ed, es, edone, part, st, n_inst,
                       tol_k, tol_phi, 1, last, G);
    hipLaunchKernelGGL(eig_apply_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks,
                       ed, es, edone, n_inst, G);
}

void launch_eig_emission(int nblocks, const InstDesc* insts, const int4* blocks,
                         const EigDesc* ed, const EigState* es, const int* edone,
                         hipStream_t s) {
    hipLaunchKernelGGL(eig_emission_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks,
                       ed, es, edone);
}

void launch_mg_fission(int n_inst, int G, int nblocks, const InstDesc* insts, const int4* blocks,
                       const EigDesc* ed, const MgDesc* md, const EigState* es,
                       const int* edone, hipStream_t s) {
    hipLaunchKernelGGL(mg_fission_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks,
                       ed, md, es, edone, n_inst, G);
}

void launch_mg_group(int n_pseudo, int G, int g, int nblocks, const InstDesc* insts,
                     const int4* blocks, const EigDesc* ed, const MgDesc* md, const int* edone,
                     int* skip, hipStream_t s) {
    hipLaunchKernelGGL(mg_source_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks,
                       ed, md, edone, n_pseudo / G, g);
    hipLaunchKernelGGL(mg_mask_kernel, dim3((n_pseudo + 255) / 256), dim3(256), 0, s, edone,
                       skip, n_pseudo, n_pseudo / G, g);
}

void launch_eig_final(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                      const EigState* es, hipStream_t s) {
    hipLaunchKernelGGL(eig_final_kernel, dim3(nblocks), dim3(kThreads), 0, s, insts, blocks,
                       es, n_inst);
}

}  // namespace mdp
