// common.h -- device-side descriptors shared by the HIP kernels and the host
// side of libmdpnop.  Internal to the library; the public ABI is mdpnop.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdp {

constexpr int kMaxDir = 512;   // directions per quadrature set

// Quadrature as the kernels see it.  Octants (2-D): 0 (+mu,+eta),
// 1 (-mu,+eta), 2 (-mu,-eta), 3 (+mu,-eta).  1-D uses octants 0 (mu > 0)
// and 1 (mu < 0).  list[o][k] is the caller's direction index.
struct DirTable {
    int M;
    int count[4];
    int list[4][kMaxDir];
    float amu[kMaxDir], aeta[kMaxDir], w[kMaxDir];   // |mu|, |eta|, weight
    float mu[kMaxDir], eta[kMaxDir];                 // signed
    int mirx[kMaxDir], miry[kMaxDir];                // mirrored across x / y faces
};

// One problem instance as every kernel sees it.
struct InstDesc {
    const float *st, *ss, *q;      // caller fields
    float *phi;                    // caller output (the iterate)
    float *Q;                      // emission sigma_s*phi + q (workspace, or
                                   // the caller's emission in a bare sweep)
    float *part;                   // P partial scalar-flux planes [P][cells]
    float *face;                   // [2 parity][4 faces][nf][M] (2-D),
                                   // [2][2][M] (1-D)
    const float *phi_init;         // warm start or nullptr
    float *snap;                   // iterate kStopStride iterations back
                                   // (error-bound stopping rule) or nullptr
    const float *ss1;              // first Legendre moment of scattering
                                   // (P1) or nullptr (isotropic)
    float *Ex, *Ey;                // P1 emission fields 3 sigma_s1 J (Ey: 2-D)
    float *partJ;                  // 2-D P1: current planes [2][P][cells]
    int dim, nx, ny, nf, cells;
    int R;                         // rows per lane segment (64, 32, 16)
    int S;                         // direction slices per octant
    int P;                         // partial planes (4*S in 2-D, M in 1-D)
    int red0, nred;                // range of reduction blocks
    float inv_dx, inv_dy;
    double dx, dy;
    int bc[4];
};

struct SweepWork {
    int inst, oct, slice, pad;
};

// Per-instance iteration state on the device.
struct IterState {
    int *done;        // 1 once converged / failed
    int *iter;        // sweeps performed
    int *status;      // 0 ok, 1 not converged, -4 non-finite
    double *resid;    // last change norm
    double *rhist;    // [n][2]: change norm of iteration l in slot l & 1
};

// Change norms (norm_kind): 0 relative L2 change, 1 max relative change,
// 2 error bound of the fixed-point iteration.  For the bound the iterate is
// compared with the one kStopStride iterations back: with
// r = ||phi_l - phi_(l-K)|| / ||phi_l|| and the observed contraction over K
// iterations rho = r_l / r_(l-K), the distance to the fixed point is about
// r rho / (1 - rho); the test stops once rho < 1 and that estimate is below
// tol, and runs only at iterations l that are multiples of K.  (Measured over
// K iterations the change stands well above the FP32 rounding floor of the
// one-iteration change, about 1e-7 relative, which would otherwise hide the
// slowly decaying error of a problem with a contraction rate near 1.)
// r_prev is INFINITY before the second test.
constexpr int kStopStride = 16;

__device__ __forceinline__ bool stop_test(double r, double r_prev, double tol, int norm_kind) {
    if (norm_kind != 2) return r < tol;
    if (r == 0.0) return true;
    if (!(r_prev < INFINITY) || !(r_prev > 0.0)) return false;
    const double rho = r / r_prev;
    if (!(rho < 1.0)) return false;
    return r * rho / (1.0 - rho) < tol;
}

// Whether iteration l (1-based) is tested, and the slot of the residual
// history its change norm goes to (the previous tested one is in the other).
__device__ __forceinline__ bool tested_iteration(int l, int norm_kind) {
    return norm_kind != 2 || l % kStopStride == 0;
}
__device__ __forceinline__ int history_slot(int l, int norm_kind) {
    return (norm_kind == 2 ? l / kStopStride : l) & 1;
}

// Convergence test of the previous iteration, run by the next sweep: every
// workgroup of an instance evaluates it from the combine kernel's FP64
// partial sums (fixed order) and leaves when the instance is finished; one
// designated workgroup records it.  pending = 0: nothing to test (the first
// sweep, or the host ran the separate finalize kernel since).  it = sweeps
// launched so far in this solve (every active instance has performed that
// many), which gives the face parity without reading the state being
// updated; it also tells whether this iteration is tested and which slot
// of the residual history its change norm goes to.
struct FinArgs {
    const double2* red;
    IterState st;
    double tol;
    int norm_kind;
    int pending;
    int it;
};

// Returns true when instance n is finished (the caller's workgroup exits).
__device__ __forceinline__ bool sweep_prologue(const InstDesc& I, int n, const FinArgs& f,
                                               bool designated) {
    if (f.st.done[n]) return true;
    if (!tested_iteration(f.it, f.norm_kind)) {
        if (designated && threadIdx.x == 0) f.st.iter[n] += 1;
        return false;
    }
    // the finalize kernel's summation order, with the loads issued 8 at a time
    double s1 = 0.0, s2 = 0.0;
    int b = 0;
    for (; b + 8 <= I.nred; b += 8) {
        double2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = f.red[I.red0 + b + j];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (f.norm_kind != 1) { s1 += v[j].x; s2 += v[j].y; }
            else s1 = fmax(s1, v[j].x);
        }
    }
    for (; b < I.nred; ++b) {
        const double2 v = f.red[I.red0 + b];
        if (f.norm_kind != 1) { s1 += v.x; s2 += v.y; }
        else s1 = fmax(s1, v.x);
    }
    double r;
    if (f.norm_kind != 1)
        r = s2 > 0.0 ? sqrt(s1 / s2) : (s1 == 0.0 ? 0.0 : INFINITY);
    else
        r = s1;
    const bool bad = !isfinite(s1) || !isfinite(s2);
    const int slot = history_slot(f.it, f.norm_kind);
    const double r_prev = f.st.rhist[2 * n + (slot ^ 1)];
    const bool conv = !bad && stop_test(r, r_prev, f.tol, f.norm_kind);
    if (designated && threadIdx.x == 0) {
        f.st.resid[n] = r;
        f.st.rhist[2 * n + slot] = r;
        f.st.iter[n] += 1;
        if (bad) {
            f.st.status[n] = -4;
            f.st.done[n] = 1;
        } else if (conv) {
            f.st.status[n] = 0;
            f.st.done[n] = 1;
        }
    }
    return bad || conv;
}

// Arguments of the persistent iteration kernel (several source iterations
// per launch: sweep, combine and convergence test, with a barrier of each
// instance's workgroups between the phases).  bar[n] counts the barrier
// arrivals of instance n over the solve (zeroed before its first launch);
// a wait that exceeds spin_limit polls sets *err and goes on, so every
// workgroup finishes whatever happens.
struct PersistArgs {
    int* bar;
    int* err;
    int spin_limit;
    int it0;          // iterations done before this launch (by every active instance)
    int k;            // iterations in this launch
    int norm_kind;
    double tol;
    double2* red;
    IterState st;
};

constexpr int kCombineThreads = 256;
constexpr int kCombineChunk = 2048;   // cells per combine block
constexpr int kXcds = 8;              // accelerator complex dies (L2 domains)

}  // namespace mdp
