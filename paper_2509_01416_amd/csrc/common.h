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
};

// Convergence test of the previous iteration, run by the next sweep: every
// workgroup of an instance evaluates it from the combine kernel's FP64
// partial sums (fixed order) and leaves when the instance is finished; one
// designated workgroup records it.  pending = 0: nothing to test (the first
// sweep, or the host ran the separate finalize kernel since).  it = sweeps
// launched so far in this solve (every active instance has performed that
// many), which gives the face parity without reading the state being
// updated.
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
    // the finalize kernel's summation order, with the loads issued 8 at a time
    double s1 = 0.0, s2 = 0.0;
    int b = 0;
    for (; b + 8 <= I.nred; b += 8) {
        double2 v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = f.red[I.red0 + b + j];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (f.norm_kind == 0) { s1 += v[j].x; s2 += v[j].y; }
            else s1 = fmax(s1, v[j].x);
        }
    }
    for (; b < I.nred; ++b) {
        const double2 v = f.red[I.red0 + b];
        if (f.norm_kind == 0) { s1 += v.x; s2 += v.y; }
        else s1 = fmax(s1, v.x);
    }
    double r;
    if (f.norm_kind == 0)
        r = s2 > 0.0 ? sqrt(s1 / s2) : (s1 == 0.0 ? 0.0 : INFINITY);
    else
        r = s1;
    const bool bad = !isfinite(s1) || !isfinite(s2);
    const bool conv = !bad && r < f.tol;
    if (designated && threadIdx.x == 0) {
        f.st.resid[n] = r;
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

constexpr int kCombineThreads = 256;
constexpr int kCombineChunk = 2048;   // cells per combine block
constexpr int kXcds = 8;              // accelerator complex dies (L2 domains)

}  // namespace mdp
