// eigen_kernels.h -- device descriptors and launchers of the outer update P
// of the one-group k-eigenvalue power iteration (internal to libmdpnop).
#pragma once

#include "common.h"

namespace mdp {

constexpr int kMaxGroups = 8;   // energy groups of a multigroup problem

// Per instance of the inner solve (one group of one problem), as the eigen
// kernels see it.
struct EigDesc {
    const float* nsf;    // nu*sigma_f (caller, cells)
    const float* phi0;   // caller's starting flux, or nullptr for a flat start
    float* S;            // the inner solve's source: nu*sigma_f*phi/k (one group), or
                         // chi_g fd + downscatter (multigroup)
    float* prev;         // last normalised iterate
    double vol;          // cell volume (dx in 1-D, dx*dy in 2-D)
};

// Multigroup data of one problem (section 5.3): fission density buffer,
// spectrum, and the scattering fields ss[h * kMaxGroups + g] (h -> g,
// nullptr = zero; only h < g are read here, the within-group h = g field is
// the inner solve's sigma_s).
struct MgDesc {
    float* fd;
    float chi[kMaxGroups];
    const float* ss[kMaxGroups * kMaxGroups];
};

// Per-problem state of the outer loop.
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

// Launchers.  n_inst problems of G groups each; the inner solve's
// instances (insts, blocks) are the pseudo-instances j = g*n_inst + i.
// Start: phi = phi0 (or 1), then normalise it (F summed over the groups),
// store it as the previous iterate and, for G = 1, form the first fission
// source with the starting k.
void launch_eig_start(int n_inst, int G, int nblocks, const InstDesc* insts, const int4* blocks,
                      const EigDesc* ed, EigState* es, int* edone, double* part,
                      hipStream_t s);
// One outer update after the inner solves: k, normalisation, change norms,
// convergence (the last outer marks every running problem finished), and
// for problems still running the next iterate (and, for G = 1, source).
void launch_eig_update(int n_inst, int G, int nblocks, const InstDesc* insts, const int4* blocks,
                       const EigDesc* ed, EigState* es, int* edone, double* part,
                       IterState st, double tol_k, double tol_phi, int last, hipStream_t s);
// Emission sigma_s u + nu_sigma_f u / k of the running instances into the
// instances' emission buffers (one sweep of the constrained variant; G = 1).
void launch_eig_emission(int nblocks, const InstDesc* insts, const int4* blocks,
                         const EigDesc* ed, const EigState* es, const int* edone,
                         hipStream_t s);
// Multigroup: the fission density of the stored iterate (once per outer).
void launch_mg_fission(int n_inst, int G, int nblocks, const InstDesc* insts, const int4* blocks,
                       const EigDesc* ed, const MgDesc* md, const EigState* es,
                       const int* edone, hipStream_t s);
// Multigroup: the source of group g and the skip mask of its inner solve.
void launch_mg_group(int n_pseudo, int G, int g, int nblocks, const InstDesc* insts,
                     const int4* blocks, const EigDesc* ed, const MgDesc* md, const int* edone,
                     int* skip, hipStream_t s);
// After the last outer: the inner solution of every valid problem scaled by
// its normalisation (F(phi) = 1).
void launch_eig_final(int n_inst, int nblocks, const InstDesc* insts, const int4* blocks,
                      const EigState* es, hipStream_t s);

}  // namespace mdp
