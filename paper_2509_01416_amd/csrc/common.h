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

constexpr int kCombineThreads = 256;
constexpr int kCombineChunk = 2048;   // cells per combine block
constexpr int kXcds = 8;              // accelerator complex dies (L2 domains)

}  // namespace mdp
