// eigen_kernels.h -- device descriptors and launchers of the outer update P
// of the one-group k-eigenvalue power iteration (internal to libmdpnop).
#pragma once

#include "common.h"

namespace mdp {

// Per instance, as the eigen kernels see it.
struct EigDesc {
    const float* nsf;    // nu*sigma_f (caller, cells)
    const float* phi0;   // caller's starting flux, or nullptr for a flat start
    float* S;            // fission emission nu*sigma_f*phi/k: the inner solve's source
    float* prev;         // last normalised iterate
    double vol;          // cell volume (dx in 1-D, dx*dy in 2-D)
};

// Per-instance state of the outer loop.
struct EigState {
    double k;       // current eigenvalue estimate
    double F;       // F(phi) = sum nu_sigma_f phi V of the stored iterate
    double scale;   // 1 / F(phi_half) of the last inner solution
    double dk;      // |k_new - k| / |k_new| of the last update
    double dphi;    // max|phi_new - phi| / max|phi_new| of the last update
    int outer;      // outer updates performed
    int inner;      // source-iteration sweeps, summed over the inner solves
    int status;     // 1 running / not converged, 0 converged, -1 invalid, -4 non-finite
    int pad;
};

// Start: phi = phi0 (or 1), then normalise it, store it as the previous
// iterate and form the first fission source with the starting k.
void launch_eig_start(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                      const EigDesc* ed, EigState* es, int* edone, double* part,
                      hipStream_t s);
// One outer update after the inner solves: k, normalisation, change norms,
// convergence (the last outer marks every running instance finished), and
// for instances still running the next fission source.
void launch_eig_update(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                       const EigDesc* ed, EigState* es, int* edone, double* part,
                       IterState st, double tol_k, double tol_phi, int last, hipStream_t s);
// Emission sigma_s u + nu_sigma_f u / k of the running instances into the
// instances' emission buffers (one sweep of the constrained variant).
void launch_eig_emission(int nblocks, const InstDesc* insts, const int4* blocks,
                         const EigDesc* ed, const EigState* es, const int* edone,
                         hipStream_t s);
// After the last outer: the inner solution of every valid instance scaled by
// its normalisation (F(phi) = 1).
void launch_eig_final(int nblocks, const InstDesc* insts, const int4* blocks,
                      const EigState* es, hipStream_t s);

}  // namespace mdp
