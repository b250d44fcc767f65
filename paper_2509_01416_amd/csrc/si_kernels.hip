// si_kernels.hip -- the non-sweep kernels of the source iteration
// (arXiv 2509.01416: the model-based iteration M of Eq. 3a/4b, realised as
// S_N source iteration in section 5.1):
//   * 1-D slab sweep (Eq. 12 with diamond differencing);
//   * argument scan (finite values, 0 <= sigma_s <= sigma_t, sigma_t > 0);
//   * initialisation of the iterate, the emission and the boundary faces;
//   * combine: phi_new = sum of the sweep's partial planes in fixed order,
//     next emission Q = sigma_s phi_new + q, FP64 change-norm partials;
//   * finalize: per-instance FP64 change norm, convergence flag;
//   * FP64 particle balance of the converged iterate.
#include <math.h>

#include "combine_dev.h"
#include "common.h"

namespace mdp {

// ------------------------------------------------------------ 1-D sweep ---
// One thread per (instance, direction); each walks its cells in upwind order
// and writes w_m psi_m to its own partial plane (P = M planes).
__global__ void sweep1d_kernel(const InstDesc* __restrict__ insts,
                               const DirTable* __restrict__ dt,
                               const int* __restrict__ done,
                               const int* __restrict__ iter, int use_faces) {
    const int n = blockIdx.x;
    if (done != nullptr && done[n]) return;
    const InstDesc& I = insts[n];
    const int M = dt->M;
    const int par = (iter != nullptr ? iter[n] : 0) & 1;
    const float* fprev = I.face + (size_t)par * 2 * M;
    float* fcur = I.face + (size_t)(par ^ 1) * 2 * M;
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        const float mu = dt->mu[m];
        const bool pos = mu > 0.f;
        const float a = 2.0f * dt->amu[m] * I.inv_dx;
        const float wm = dt->w[m];
        const int fin = pos ? 0 : 1, fout = pos ? 1 : 0;
        float in = (use_faces && I.bc[fin] == 1) ? fprev[fin * M + dt->mirx[m]] : 0.f;
        float* part = I.part + (size_t)m * I.cells;
        const int nx = I.nx;
        const float* Ex = I.Ex;   // P1 emission 3 sigma_s1 J, or none
        for (int ii = 0; ii < nx; ++ii) {
            const int i = pos ? ii : nx - 1 - ii;
            const float qm = Ex != nullptr ? fmaf(mu, Ex[i], I.Q[i]) : I.Q[i];
            const float psi = fmaf(a, in, qm) * __builtin_amdgcn_rcpf(I.st[i] + a);
            in = psi + psi - in;
            part[i] = wm * psi;
        }
        fcur[fout * M + m] = in;
    }
}

// ------------------------------------------------------- argument scan ---
// flags[n] bit 0: a non-finite value; bit 1: sigma_t <= 0, sigma_s < 0 or
// sigma_s > sigma_t.  samax[n] = max(sigma_t - sigma_s).
// Stage 1, one workgroup per reduction block: invalid-value flags (bit 0
// non-finite, bit 1 sigma_t <= 0 or sigma_s outside [0, sigma_t]) and the
// largest sigma_a over the block's cells.  OR and max are exact, so the
// per-instance result does not depend on the order.
__global__ void __launch_bounds__(256)
scan_part_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                 double* __restrict__ part) {
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0) return;
    const InstDesc& I = insts[bi.x];
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    int bad = 0;
    float mx = 0.f;
    for (int c = bi.y + (int)threadIdx.x; c < c1; c += blockDim.x) {
        const float st = I.st[c], ss = I.ss[c], q = I.q[c];
        if (!isfinite(st) || !isfinite(ss) || !isfinite(q)) bad |= 1;
        if (I.phi_init != nullptr && !isfinite(I.phi_init[c])) bad |= 1;
        if (!(st > 0.f) || ss < 0.f || ss > st) bad |= 2;
        if (I.ss1 != nullptr) {   // P1: |sigma_s1| <= sigma_s (mean cosine in [-1, 1])
            const float s1 = I.ss1[c];
            if (!isfinite(s1)) bad |= 1;
            else if (fabsf(s1) > ss) bad |= 2;
        }
        mx = fmaxf(mx, st - ss);
    }
    __shared__ int sbad[256];
    __shared__ float smx[256];
    sbad[threadIdx.x] = bad;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sbad[threadIdx.x] |= sbad[threadIdx.x + h];
            smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * bi.z + 0] = (double)sbad[0];
        part[3 * bi.z + 1] = (double)smx[0];
    }
}

// Stage 2, one thread per instance.
__global__ void scan_fin_kernel(const InstDesc* __restrict__ insts,
                                const double* __restrict__ part, int n_inst,
                                int* __restrict__ flags, float* __restrict__ samax) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_inst) return;
    const InstDesc& I = insts[n];
    int bad = 0;
    float mx = 0.f;
    for (int b = 0; b < I.nred; ++b) {
        bad |= (int)part[3 * (size_t)(I.red0 + b)];
        mx = fmaxf(mx, (float)part[3 * (size_t)(I.red0 + b) + 1]);
    }
    flags[n] = bad;
    samax[n] = mx;
}

// ------------------------------------------------------------- init ------
// Grid: one block per reduction block (instance, first cell, slot).
__global__ void init_cells_kernel(const InstDesc* __restrict__ insts,
                                  const int4* __restrict__ blocks,
                                  const int* __restrict__ skip) {
    const int4 bi = blocks[blockIdx.x];
    if (bi.x < 0 || (skip != nullptr && skip[bi.x])) return;
    const InstDesc& I = insts[bi.x];
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    for (int c = bi.y + threadIdx.x; c < c1; c += blockDim.x) {
        const float p = I.phi_init != nullptr ? I.phi_init[c] : 0.f;
        I.phi[c] = p;
        I.Q[c] = fmaf(I.ss[c], p, I.q[c]);
        if (I.snap != nullptr) I.snap[c] = p;
        if (I.Ex != nullptr) I.Ex[c] = 0.f;   // no current before the first sweep
        if (I.Ey != nullptr) I.Ey[c] = 0.f;
    }
}

// Faces of parity 0: isotropic at the adjacent cell's initial flux (warm
// start) or zero.  One workgroup per reduction block, each taking an even
// share of its instance's face entries; the instance's first block also
// resets the iteration state.  An instance with skip[n] set keeps its
// fields, faces and sweep count and is only marked done, so the sweeps pass
// it by.
__global__ void __launch_bounds__(256)
init_faces_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                  const DirTable* __restrict__ dt, IterState st, const int* __restrict__ skip) {
    const int4 bi = blocks[blockIdx.x];
    const int n = bi.x;
    if (n < 0) return;
    const InstDesc& I = insts[n];
    const int M = dt->M;
    const int j = bi.z - I.red0;
    if (skip != nullptr && skip[n]) {
        if (j == 0 && threadIdx.x == 0) st.done[n] = 1;
        return;
    }
    if (j == 0 && threadIdx.x == 0) {
        st.done[n] = 0;
        st.iter[n] = 0;
        st.status[n] = 1;
        st.resid[n] = INFINITY;
        st.rhist[2 * n] = INFINITY;
        st.rhist[2 * n + 1] = INFINITY;
    }
    if (I.dim == 1) {
        const int total = 2 * M;
        const int e0 = (int)((long long)total * j / I.nred);
        const int e1 = (int)((long long)total * (j + 1) / I.nred);
        for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
            const int f = e / M;
            float v = 0.f;
            if (I.phi_init != nullptr) v = I.phi_init[f == 0 ? 0 : I.nx - 1];
            I.face[e] = v;
        }
        return;
    }
    const int nf = I.nf;
    const int total = 4 * nf * M;
    const int e0 = (int)((long long)total * j / I.nred);
    const int e1 = (int)((long long)total * (j + 1) / I.nred);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
        const int f = e / (nf * M);
        const int kk = (e / M) % nf;
        float v = 0.f;
        if (I.phi_init != nullptr) {
            const int len = f < 2 ? I.ny : I.nx;
            if (kk < len) {
                int c;
                if (f == 0) c = kk * I.nx;
                else if (f == 1) c = kk * I.nx + I.nx - 1;
                else if (f == 2) c = kk;
                else c = (I.ny - 1) * I.nx + kk;
                v = I.phi_init[c];
            }
        }
        I.face[e] = v;
    }
}

// ------------------------------------------------------------ combine ----
// One workgroup per block of kCombineChunk cells (combine_dev.h).
__global__ void __launch_bounds__(kCombineThreads)
combine_kernel(const InstDesc* __restrict__ insts,
               const int4* __restrict__ blocks, const int* __restrict__ done,
               double2* __restrict__ red, int mode, int norm_kind,
               const DirTable* __restrict__ dt) {
    const int4 bi = blocks[blockIdx.x];
    const int n = bi.x;
    if (n < 0) return;
    if (done != nullptr && done[n]) return;
    __shared__ double r1[kCombineThreads], r2[kCombineThreads];
    combine_block(insts[n], bi.y, bi.z, red, mode, norm_kind, dt, (int)threadIdx.x,
                  kCombineThreads, r1, r2);
}

// ----------------------------------------------------------- finalize ----
__global__ void finalize_kernel(const InstDesc* __restrict__ insts,
                                const double2* __restrict__ red, IterState st,
                                int n_inst, double tol, int norm_kind) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_inst || st.done[n]) return;
    const InstDesc& I = insts[n];
    const int l = st.iter[n] + 1;   // the iteration tested here
    if (!tested_iteration(l, norm_kind)) {
        st.iter[n] = l;
        return;
    }
    double s1 = 0.0, s2 = 0.0;
    for (int b = 0; b < I.nred; ++b) {
        const double2 v = red[I.red0 + b];
        if (norm_kind != 1) { s1 += v.x; s2 += v.y; }
        else s1 = fmax(s1, v.x);
    }
    double r;
    if (norm_kind != 1)
        r = s2 > 0.0 ? sqrt(s1 / s2) : (s1 == 0.0 ? 0.0 : INFINITY);
    else
        r = s1;
    const int slot = history_slot(l, norm_kind);
    const double r_prev = st.rhist[2 * n + (slot ^ 1)];
    st.resid[n] = r;
    st.rhist[2 * n + slot] = r;
    st.iter[n] = l;
    if (!isfinite(s1) || !isfinite(s2)) {
        st.status[n] = -4;
        st.done[n] = 1;
    } else if (stop_test(r, r_prev, tol, norm_kind)) {
        st.status[n] = 0;
        st.done[n] = 1;
    }
}

// ------------------------------------------------------------ balance ----
// bal[n] = {sum q V, sum sigma_a phi V, leakage} in FP64 for the last sweep.
// Stage 1, one workgroup per reduction block (kCombineChunk cells of one
// instance): FP64 sums of q V and sigma_a phi V over the block's cells and
// the leakage of its share of the instance's boundary-face entries (the
// entries are split evenly over the instance's blocks).
__global__ void __launch_bounds__(256)
balance_part_kernel(const InstDesc* __restrict__ insts, const int4* __restrict__ blocks,
                    const DirTable* __restrict__ dt, const int* __restrict__ iter,
                    double* __restrict__ part) {
    const int4 bi = blocks[blockIdx.x];
    const int n = bi.x;
    if (n < 0) return;
    const InstDesc& I = insts[n];
    const int M = dt->M;
    const double V = I.dx * I.dy;
    double sq = 0.0, sa = 0.0, lk = 0.0;
    const int c1 = min(bi.y + kCombineChunk, I.cells);
    for (int c = bi.y + (int)threadIdx.x; c < c1; c += blockDim.x) {
        sq += (double)I.q[c] * V;
        sa += ((double)I.st[c] - (double)I.ss[c]) * (double)I.phi[c] * V;
    }
    const int it = iter[n];
    const int pc = it & 1, pp = (it + 1) & 1;   // current / previous parity
    const int j = bi.z - I.red0;                // this block's rank in the instance
    if (I.dim == 1) {
        const int total = 2 * M;
        const int e0 = (int)((long long)total * j / I.nred);
        const int e1 = (int)((long long)total * (j + 1) / I.nred);
        const float* fc = I.face + (size_t)pc * 2 * M;
        const float* fp = I.face + (size_t)pp * 2 * M;
        for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
            const int f = e / M, m = e - f * M;
            const double on = f == 0 ? -(double)dt->mu[m] : (double)dt->mu[m];
            double psi;
            if (on > 0.0) psi = fc[f * M + m];
            else psi = I.bc[f] == 1 ? fp[f * M + dt->mirx[m]] : 0.0;
            lk += (double)dt->w[m] * on * psi;
        }
    } else {
        const int nf = I.nf;
        const size_t fs = (size_t)4 * nf * M;
        const float* fc = I.face + (size_t)pc * fs;
        const float* fp = I.face + (size_t)pp * fs;
        const int total = 4 * nf * M;
        const int e0 = (int)((long long)total * j / I.nred);
        const int e1 = (int)((long long)total * (j + 1) / I.nred);
        for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
            const int f = e / (nf * M);
            const int kk = (e / M) % nf;
            const int m = e % M;
            const int len = f < 2 ? I.ny : I.nx;
            if (kk >= len) continue;
            double on;
            if (f == 0) on = -(double)dt->mu[m];
            else if (f == 1) on = (double)dt->mu[m];
            else if (f == 2) on = -(double)dt->eta[m];
            else on = (double)dt->eta[m];
            const double A = f < 2 ? I.dy : I.dx;
            double psi;
            if (on > 0.0) {
                psi = fc[e];
            } else if (I.bc[f] == 1) {
                const int mm = f < 2 ? dt->mirx[m] : dt->miry[m];
                psi = fp[((size_t)f * nf + kk) * M + mm];
            } else {
                psi = 0.0;
            }
            lk += (double)dt->w[m] * on * psi * A;
        }
    }
    __shared__ double r[3][256];
    r[0][threadIdx.x] = sq;
    r[1][threadIdx.x] = sa;
    r[2][threadIdx.x] = lk;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) r[k][threadIdx.x] += r[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * bi.z + 0] = r[0][0];
        part[3 * bi.z + 1] = r[1][0];
        part[3 * bi.z + 2] = r[2][0];
    }
}

// Stage 2, one thread per instance: the block partials summed in block order.
__global__ void balance_fin_kernel(const InstDesc* __restrict__ insts,
                                   const double* __restrict__ part, int n_inst,
                                   double* __restrict__ bal) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= n_inst) return;
    const InstDesc& I = insts[n];
    double sq = 0.0, sa = 0.0, lk = 0.0;
    for (int b = 0; b < I.nred; ++b) {
        const double* v = part + 3 * (size_t)(I.red0 + b);
        sq += v[0];
        sa += v[1];
        lk += v[2];
    }
    bal[3 * n + 0] = sq;
    bal[3 * n + 1] = sa;
    bal[3 * n + 2] = lk;
}

// ------------------------------------------------------------ launchers --
void launch_sweep1d(int n_inst, const InstDesc* insts, const DirTable* dt,
                    const int* done, const int* iter, int use_faces, int M,
                    hipStream_t s) {
    const int th = M <= 64 ? 64 : (M <= 256 ? 256 : 1024);
    hipLaunchKernelGGL(sweep1d_kernel, dim3(n_inst), dim3(th), 0, s, insts, dt,
                       done, iter, use_faces);
}

void launch_scan(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                 double* part, int* flags, float* samax, hipStream_t s) {
    hipLaunchKernelGGL(scan_part_kernel, dim3(nblocks), dim3(256), 0, s, insts, blocks, part);
    hipLaunchKernelGGL(scan_fin_kernel, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, part,
                       n_inst, flags, samax);
}

void launch_init(int n_inst, int nblocks, const InstDesc* insts,
                 const int4* blocks, const DirTable* dt, IterState st,
                 const int* skip, hipStream_t s) {
    hipLaunchKernelGGL(init_cells_kernel, dim3(nblocks), dim3(kCombineThreads), 0,
                       s, insts, blocks, skip);
    hipLaunchKernelGGL(init_faces_kernel, dim3(nblocks), dim3(256), 0, s, insts, blocks,
                       dt, st, skip);
}

void launch_combine(int nblocks, const InstDesc* insts, const int4* blocks,
                    const int* done, double2* red, int mode, int norm_kind,
                    hipStream_t s, const DirTable* dt) {
    hipLaunchKernelGGL(combine_kernel, dim3(nblocks), dim3(kCombineThreads), 0, s,
                       insts, blocks, done, red, mode, norm_kind, dt);
}

void launch_finalize(int n_inst, const InstDesc* insts, const double2* red,
                     IterState st, double tol, int norm_kind, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3((n_inst + 63) / 64), dim3(64), 0, s,
                       insts, red, st, n_inst, tol, norm_kind);
}

void launch_balance(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                    const DirTable* dt, const int* iter, double* part, double* bal,
                    hipStream_t s) {
    hipLaunchKernelGGL(balance_part_kernel, dim3(nblocks), dim3(256), 0, s, insts, blocks, dt,
                       iter, part);
    hipLaunchKernelGGL(balance_fin_kernel, dim3((n_inst + 63) / 64), dim3(64), 0, s, insts, part,
                       n_inst, bal);
}

}  // namespace mdp
