// combine_dev.h -- the combine step of the source iteration on one block of
// kCombineChunk cells (internal): the fixed-order sum of an instance's
// partial scalar-flux planes, the next emission and the FP64 change-norm
// partials of the block.  Used by combine_kernel (one workgroup per block)
// and by the persistent iteration kernel (a sweep workgroup takes a share
// of its instance's blocks), with the same arithmetic.
#pragma once

#include <math.h>

#include "common.h"

namespace mdp {

// ------------------------------------------------------------ combine ----
// mode 0: source-iteration update (phi, Q, change-norm partials);
// mode 1: bare sweep (phi = sum of planes);
// mode 2: source-iteration update with the norm partials of the change
//         against the snapshot, which then takes phi_new (error-bound rule,
//         tested iterations);
// mode 3: source-iteration update without norm partials (error-bound rule,
//         untested iterations).  The planes of a cell are summed
// in plane order; with cells % 4 == 0 four cells move per 16-byte access.
struct CellAcc {
    double s1 = 0.0, s2 = 0.0;
};

__device__ __forceinline__ void combine_norm(float old, float s, int norm_kind, CellAcc& a) {
    const double d = (double)s - (double)old;
    if (norm_kind != 1) {
        a.s1 += d * d;
        a.s2 += (double)s * (double)s;
    } else {
        const double as = fabs((double)s);
        const double rel = as > 0.0 ? fabs(d) / as : (d != 0.0 ? INFINITY : 0.0);
        a.s1 = fmax(a.s1, rel);
    }
}

// P1 emission of the next sweep from the current of this one: the 1-D
// planes are per direction (w psi), so J = sum_m mu_m plane_m; the 2-D
// sweep writes current planes beside the flux planes.  Fixed order.
__device__ __forceinline__ void combine_p1(const InstDesc& I, int c, const DirTable* dt) {
    if (I.dim == 1) {
        const float* pp = I.part + c;
        float j = 0.f;
        for (int p = 0; p < I.P; ++p) j = fmaf(dt->mu[p], pp[(size_t)p * I.cells], j);
        I.Ex[c] = I.ss1 != nullptr ? 3.0f * I.ss1[c] * j : 0.f;
        return;
    }
    const float* px = I.partJ + c;
    const float* py = I.partJ + (size_t)I.P * I.cells + c;
    float jx = 0.f, jy = 0.f;
    for (int p = 0; p < I.P; ++p) {
        jx += px[(size_t)p * I.cells];
        jy += py[(size_t)p * I.cells];
    }
    const float k = I.ss1 != nullptr ? 3.0f * I.ss1[c] : 0.f;
    I.Ex[c] = k * jx;
    I.Ey[c] = k * jy;
}

__device__ __forceinline__ void combine_cell(const InstDesc& I, int c, float s,
                                             int mode, int norm_kind, CellAcc& a) {
    if (mode == 1) {
        I.phi[c] = s;
        return;
    }
    // the previous flux only where a norm is taken (not on untested
    // iterations of the error-bound rule)
    const float old = mode == 3 ? 0.f : (mode == 2 ? I.snap[c] : I.phi[c]);
    I.phi[c] = s;
    I.Q[c] = fmaf(I.ss[c], s, I.q[c]);
    if (mode == 2) I.snap[c] = s;
    if (mode != 3) combine_norm(old, s, norm_kind, a);
}

// One block of instance I: cells [c0, c0 + kCombineChunk), norm partials
// into red[z].  The work is that of kCombineThreads virtual threads (the
// cells each one owns and the order it accumulates them in, then a tree
// over the virtual threads), carried by the nthr threads of the workgroup
// (virtual thread v on thread v mod nthr), so that any workgroup size gives
// the same sums as the combine kernel's.  Every thread of the workgroup
// must call it (the reduction synchronises the workgroup); r1, r2 are
// kCombineThreads doubles of LDS each.
__device__ __forceinline__ void combine_block(const InstDesc& I, int c0, int z,
                                              double2* __restrict__ red, int mode,
                                              int norm_kind, const DirTable* __restrict__ dt,
                                              int tid, int nthr, double* r1, double* r2) {
    const int cells = I.cells, P = I.P;
    const int c1 = min(c0 + kCombineChunk, cells);
    const bool al16 = ((reinterpret_cast<uintptr_t>(I.phi) | reinterpret_cast<uintptr_t>(I.ss) |
                        reinterpret_cast<uintptr_t>(I.q) | reinterpret_cast<uintptr_t>(I.Q) |
                        reinterpret_cast<uintptr_t>(I.snap)) &
                       15) == 0;
    const bool p1 = I.Ex != nullptr && mode != 1;
    const bool vec = (cells & 3) == 0 && (al16 || mode == 1) && !p1 &&
                     (reinterpret_cast<uintptr_t>(I.phi) & 15) == 0;
    for (int v = tid; v < kCombineThreads; v += nthr) {
        CellAcc acc;
        if (vec) {
            // four cells per thread: every plane load of a thread in flight
            // at once (8 at a time), the cell fields read and written as float4
            const float4* pl = reinterpret_cast<const float4*>(I.part);
            const int q4 = cells >> 2;
            for (int c = c0 + 4 * v; c < c1; c += 4 * kCombineThreads) {
                const float4* pp = pl + (c >> 2);
                float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
                int p = 0;
                for (; p + 8 <= P; p += 8) {
                    float4 w[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) w[j] = pp[(size_t)(p + j) * q4];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        s.x += w[j].x; s.y += w[j].y; s.z += w[j].z; s.w += w[j].w;
                    }
                }
                for (; p < P; ++p) {
                    const float4 w = pp[(size_t)p * q4];
                    s.x += w.x; s.y += w.y; s.z += w.z; s.w += w.w;
                }
                float4* phi4 = reinterpret_cast<float4*>(I.phi) + (c >> 2);
                if (mode == 1) {
                    *phi4 = s;
                    continue;
                }
                // the previous flux only where a norm is taken
                float4 old = make_float4(0.f, 0.f, 0.f, 0.f);
                if (mode != 3)
                    old = mode == 2 ? reinterpret_cast<const float4*>(I.snap)[c >> 2] : *phi4;
                const float4 ss = reinterpret_cast<const float4*>(I.ss)[c >> 2];
                const float4 qq = reinterpret_cast<const float4*>(I.q)[c >> 2];
                *phi4 = s;
                reinterpret_cast<float4*>(I.Q)[c >> 2] =
                    make_float4(fmaf(ss.x, s.x, qq.x), fmaf(ss.y, s.y, qq.y),
                                fmaf(ss.z, s.z, qq.z), fmaf(ss.w, s.w, qq.w));
                if (mode == 2) reinterpret_cast<float4*>(I.snap)[c >> 2] = s;
                if (mode == 3) continue;
                combine_norm(old.x, s.x, norm_kind, acc);
                combine_norm(old.y, s.y, norm_kind, acc);
                combine_norm(old.z, s.z, norm_kind, acc);
                combine_norm(old.w, s.w, norm_kind, acc);
            }
        } else {
            for (int c = c0 + v; c < c1; c += kCombineThreads) {
                const float* pp = I.part + c;
                float s = 0.f;
                for (int p = 0; p < P; ++p) s += pp[(size_t)p * cells];
                combine_cell(I, c, s, mode, norm_kind, acc);
                if (p1) combine_p1(I, c, dt);
            }
        }
        if (mode != 1 && mode != 3) {
            r1[v] = acc.s1;
            r2[v] = acc.s2;
        }
    }
    if (mode == 1 || mode == 3) return;
    __syncthreads();
    for (int h = kCombineThreads / 2; h > 0; h >>= 1) {
        for (int v = tid; v < h; v += nthr) {
            if (norm_kind != 1) {
                r1[v] += r1[v + h];
                r2[v] += r2[v + h];
            } else {
                r1[v] = fmax(r1[v], r1[v + h]);
            }
        }
        __syncthreads();
    }
    if (tid == 0) red[z] = make_double2(r1[0], r2[0]);
}


}  // namespace mdp
