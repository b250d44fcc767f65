// sweep2d.hip -- diamond-difference transport sweep in x-y geometry for a
// batch of instances of uneven size (the transport sweep of the S_N source
// iteration, arXiv 2509.01416 section 5.1 after Eq. 20), fused with the
// quadrature reduction to the scalar flux (Eq. 17).
//
// Per direction m and cell, with a = 2|mu|/dx, b = 2|eta|/dy:
//     psi = (Q + a psi_x_in + b psi_y_in) / (sigma_t + a + b)
//     psi_x_out = 2 psi - psi_x_in,   psi_y_out = 2 psi - psi_y_in
//     phi += w_m psi
//
// Work decomposition (one workgroup per (instance, octant, direction slice)):
//   * a lane owns one row of cells and walks it in the octant's x order; a
//     wave holds 64/R segments of R lanes, all on the same R rows, each with
//     its own D directions;
//   * lane r of a segment is one step behind lane r-1, so the y-face flux it
//     needs was produced by lane r-1 on the previous step and arrives by a
//     lane shuffle (the diagonal wavefront of the row block);
//   * when a lane finishes its row it continues with the row R above it, so
//     a segment streams through ceil(ny/R) row blocks without pipeline
//     drain; the first lane of a block receives the y-face flux of the last
//     lane of the previous block through a small LDS ring (written nx-R+1
//     steps earlier, R <= nx);
//   * the W waves of the workgroup process identical cells at identical
//     steps, each for its own directions; their partial scalar fluxes are
//     combined in LDS every KB steps, in fixed wave order, and one partial
//     plane per (octant, slice) is written to HBM.  The planes are summed in
//     fixed order by the combine kernel, so the result is bitwise
//     reproducible (no floating-point atomics).
//   * angular fluxes never leave the chip except on boundary faces, which are
//     stored for reflective inflow (lagged one iteration) and leakage.
#include "common.h"

namespace mdp {

template <int D>
__global__ void __launch_bounds__(1024)
sweep2d_kernel(const InstDesc* __restrict__ insts,
               const SweepWork* __restrict__ work,
               const DirTable* __restrict__ dt, const int* __restrict__ done,
               const int* __restrict__ iter, int KB, int use_faces) {
    extern __shared__ float smem[];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int W = blockDim.x >> 6;
    const SweepWork wk = work[blockIdx.x];
    const int n = wk.inst;
    if (done != nullptr && done[n]) return;   // uniform over the workgroup
    const InstDesc& I = insts[n];
    const int R = I.R, nseg = 64 / R, seg = lane / R, r = lane - seg * R;
    const int o = wk.oct;
    const bool xpos = (o == 0 || o == 3), ypos = (o == 0 || o == 1);
    const int nx = I.nx, ny = I.ny, nf = I.nf, M = dt->M;
    const int par = (iter != nullptr ? iter[n] : 0) & 1;
    const size_t fstride = (size_t)4 * nf * M;
    const float* __restrict__ fprev = I.face + (size_t)par * fstride;
    float* __restrict__ fcur = I.face + (size_t)(par ^ 1) * fstride;
    const int fxin = xpos ? 0 : 1, fxout = xpos ? 1 : 0;
    const int fyin = ypos ? 2 : 3, fyout = ypos ? 3 : 2;
    const bool rx = use_faces && I.bc[fxin] == 1;
    const bool ry = use_faces && I.bc[fyin] == 1;

    float a[D], b[D], c[D], w[D];
    int mi[D], mxr[D], myr[D];
    const int nd = dt->count[o];
    const int base = wk.slice * (W * nseg * D) + (wv * nseg + seg) * D;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int kk = base + d;
        if (kk < nd) {
            const int m = dt->list[o][kk];
            a[d] = 2.0f * dt->amu[m] * I.inv_dx;
            b[d] = 2.0f * dt->aeta[m] * I.inv_dy;
            w[d] = dt->w[m];
            mi[d] = m;
            mxr[d] = dt->mirx[m];
            myr[d] = dt->miry[m];
        } else {
            a[d] = 0.f; b[d] = 0.f; w[d] = 0.f;
            mi[d] = -1; mxr[d] = 0; myr[d] = 0;
        }
        c[d] = a[d] + b[d];
    }

    float* pbuf = smem;
    float* ring = smem + 2 * KB * W * 64 + (size_t)((wv * nseg + seg) * D) * nx;
    const int nblk = (ny + R - 1) / R;
    const int T = nblk * nx + R - 1;
    const float* __restrict__ St = I.st;
    const float* __restrict__ Qb = I.Q;
    float* __restrict__ part = I.part + (size_t)(o * I.S + wk.slice) * I.cells;

    float xin[D], yo[D];
#pragma unroll
    for (int d = 0; d < D; ++d) { xin[d] = 0.f; yo[d] = 0.f; }

    int ip = -r, k = 0;   // position of this lane: cell ip of row block k
    for (int t0 = 0, blkno = 0; t0 < T; t0 += KB, ++blkno) {
        const int half = blkno & 1;
        const int tend = min(KB, T - t0);
        for (int tt = 0; tt < tend; ++tt) {
            const bool act = ip >= 0 && k < nblk;
            const int jp = k * R + r;
            const bool valid = act && jp < ny;
            const int i = xpos ? ip : nx - 1 - ip;
            const int j = ypos ? jp : ny - 1 - jp;
            const int cell = j * nx + i;
            float st = 1.f, q = 0.f;
            if (valid) { st = St[cell]; q = Qb[cell]; }
            float yi[D];
#pragma unroll
            for (int d = 0; d < D; ++d) yi[d] = __shfl_up(yo[d], 1, 64);
            if (r == 0 && act) {
                if (k == 0) {
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        yi[d] = (ry && mi[d] >= 0)
                                    ? fprev[((size_t)fyin * nf + i) * M + myr[d]]
                                    : 0.f;
                } else {
#pragma unroll
                    for (int d = 0; d < D; ++d) yi[d] = ring[d * nx + ip];
                }
            }
            if (ip == 0) {
#pragma unroll
                for (int d = 0; d < D; ++d)
                    xin[d] = (valid && rx && mi[d] >= 0)
                                 ? fprev[((size_t)fxin * nf + j) * M + mxr[d]]
                                 : 0.f;
            }
            float acc = 0.f;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const float rc = __builtin_amdgcn_rcpf(st + c[d]);
                const float psi = fmaf(a[d], xin[d], fmaf(b[d], yi[d], q)) * rc;
                const float p2 = psi + psi;
                xin[d] = p2 - xin[d];
                yo[d] = p2 - yi[d];
                acc = fmaf(w[d], psi, acc);
            }
            for (int off = R; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
            if (seg == 0) pbuf[((half * KB + tt) * W + wv) * 64 + r] = acc;
            if (valid) {
                if (r == R - 1 && k + 1 < nblk) {
#pragma unroll
                    for (int d = 0; d < D; ++d) ring[d * nx + ip] = yo[d];
                }
                if (ip == nx - 1) {
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        if (mi[d] >= 0)
                            fcur[((size_t)fxout * nf + j) * M + mi[d]] = xin[d];
                }
                if (jp == ny - 1) {
#pragma unroll
                    for (int d = 0; d < D; ++d)
                        if (mi[d] >= 0)
                            fcur[((size_t)fyout * nf + i) * M + mi[d]] = yo[d];
                }
            }
            // keep the ring write of this step ahead of later ring reads
            __builtin_amdgcn_wave_barrier();
            ++ip;
            if (ip == nx) { ip = 0; ++k; }
        }
        __syncthreads();
        // fixed-order combine of the waves' partial fluxes for this block
        const int nout = tend * R;
        for (int e = threadIdx.x; e < nout; e += blockDim.x) {
            const int rr = e / tend;
            const int t2 = e - rr * tend;
            const int u = t0 + t2 - rr;
            if (u < 0) continue;
            const int kk = u / nx;
            if (kk >= nblk) continue;
            const int ip2 = u - kk * nx;
            const int jp2 = kk * R + rr;
            if (jp2 >= ny) continue;
            const int i2 = xpos ? ip2 : nx - 1 - ip2;
            const int j2 = ypos ? jp2 : ny - 1 - jp2;
            const float* pb = pbuf + (size_t)(half * KB + t2) * W * 64 + rr;
            float s = 0.f;
            for (int v = 0; v < W; ++v) s += pb[v * 64];
            part[j2 * nx + i2] = s;
        }
    }
}

// Host launcher; returns false for an unsupported D.
bool launch_sweep2d(int D, int nwork, int W, int KB, size_t lds_bytes,
                    const InstDesc* insts, const SweepWork* work,
                    const DirTable* dt, const int* done, const int* iter,
                    int use_faces, hipStream_t s) {
    dim3 grid(nwork), block(64 * W);
    switch (D) {
#define MDP_CASE(DD)                                                          \
    case DD:                                                                  \
        hipLaunchKernelGGL(sweep2d_kernel<DD>, grid, block, lds_bytes, s,     \
                           insts, work, dt, done, iter, KB, use_faces);       \
        return true;
        MDP_CASE(1)
        MDP_CASE(2)
        MDP_CASE(3)
        MDP_CASE(4)
        MDP_CASE(5)
        MDP_CASE(6)
        MDP_CASE(9)
        MDP_CASE(10)
#undef MDP_CASE
        default:
            return false;
    }
}

size_t sweep2d_lds_bytes(int W, int KB, int D, int max_nseg_nx) {
    return sizeof(float) * ((size_t)2 * KB * W * 64 + (size_t)W * D * max_nseg_nx);
}

}  // namespace mdp
