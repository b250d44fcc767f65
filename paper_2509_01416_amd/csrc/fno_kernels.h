// fno_kernels.h -- launch interface of the network kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

namespace mdp {

// A strided view of a batched matrix: element (g, r, c) sits at
//   p + split(g, b_ls, sb_hi, sb_lo) + split(r, ...) + split(c, ...)
// with split(i, ls, hi, lo) = (i >> ls) * hi + (i & (2^ls - 1)) * lo, or
// i * lo when ls >= 31 (no split).
struct View {
    float* p = nullptr;
    long long sb_hi = 0, sb_lo = 0;
    int b_ls = 31;
    long long sr_hi = 0, sr_lo = 0;
    int r_ls = 31;
    long long sc_hi = 0, sc_lo = 0;
    int c_ls = 31;
};

// The lift evaluated where its output is read (inference): channel c of
// sample b at cell (ix, iy) of the 64 x 64 grid is W0[c] in + W0[32 + c] x
// + W0[64 + c] y + b0[c] with x = (ix + 1/2) / 64, y = (iy + 1/2) / 64,
// exactly as lift_kernel computes and stores it.  in == nullptr: read the
// stored lift instead.
struct LiftArgs {
    const float* in = nullptr;   // [B][64 * 64] network input
    const float* W0 = nullptr;   // [3][32]
    const float* b0 = nullptr;   // [32]
};

struct GemmArgs {
    int M = 0, N = 0, K = 0, G = 1;
    View A, B, C;
    float alpha = 1.f;
    int accumulate = 0;
    const float* bias_row = nullptr;   // added per output row m
    const float* bias_col = nullptr;   // added per output column n
    int ksplit = 1;
    float* partial = nullptr;          // [ksplit][G][M][N] when ksplit > 1
    int f32 = 0;                       // FP32 operands instead of BF16
    float* gelu_out = nullptr;         // also write gelu(C) at C's offsets
    float* relu_out = nullptr;         // also write max(C, 0) at C's offsets
};

bool launch_gemm(const GemmArgs& a, hipStream_t s);
void launch_lift(const float* in, const float* W0, const float* b0, float* out, int B,
                 int n, int C, hipStream_t s);
void launch_gelu_back(const float* z, const float* gv, float* gz, long long n, hipStream_t s);
void launch_mix(const float* X, const float* R, float* Y, int B, int C, int m, hipStream_t s);
void launch_mix_back_x(const float* gY, const float* R, float* gX, int B, int C, int m,
                       hipStream_t s);
void launch_mix_back_w(const float* X, const float* gY, float* gR, int B, int C, int m,
                       hipStream_t s);
// Pointwise path of a Fourier layer for C = 32 channels and P % 64 == 0.
void launch_pointwise(const float* W, const float* v, const float* bias, float* z, float* vn,
                      int B, int P, int store_z, int f32, hipStream_t s,
                      const LiftArgs& lift = LiftArgs{});
// Truncated 2-D DFT of G fields (64 x 64, 12 x 24 retained modes) and its
// inverse, each in one kernel (layouts as the batched GEMM path).
size_t spec_image_bytes();   // FP32 + BF16 LDS images of the DFT matrices
void launch_stage_spec(const float* FxT, const float* Fy, const float* Gy, const float* Gx,
                       void* img, hipStream_t s);
void launch_spec_fwd(const float* v, const void* img, float* X, int G, int f32, hipStream_t s,
                     const LiftArgs& lift = LiftArgs{});
void launch_spec_inv(const float* Y, const void* img, float* U, int G, int f32, hipStream_t s);
// Projection head in one kernel (width 32, 128 hidden units only).
// the last pointwise layer and the projection head in one kernel (32
// channels, 128 hidden units): z (the spectral path on entry) becomes
// W^T v + z + bias, stored if store_z; out and, if h_out, the hidden layer
void launch_pointwise_proj(const float* W, const float* v, const float* bias, float* z,
                           int store_z, const float* P1, const float* c1, const float* P2,
                           const float* c2, float* out, float* h_out, int B, int P, int f32,
                           hipStream_t s);
void launch_proj_fused(const float* v, const float* P1, const float* c1, const float* P2,
                       const float* c2, float* out, float* h_out, int B, int P, int f32,
                       hipStream_t s);
void launch_proj_back(const float* h, const float* P2, const float* gout, float* gh, int B,
                      int P, int K, hipStream_t s);
// scratch (device, >= 4 * max(R, C) * B * P / 1024 floats) selects the
// two-stage parallel form; nullptr the single-stage one.
void launch_row_reduce(const float* x, const float* w, float* out, int B, int R, int P,
                       int mode, int accumulate, float* scratch, hipStream_t s);
void launch_lift_back(const float* in, const float* gv, float* gW0, float* gb0, int B, int n,
                      int C, float* scratch, hipStream_t s);
int launch_mse(const float* out, const float* t, float* gout, double* partial, long long n,
               hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s);
void launch_recast_input(const float* S, const float* sa, const float* phi, float sa_star,
                         float* in, float* scale, const int* active, int B, int P,
                         hipStream_t s);
// Per-instance state of the recast loop's stopping and divergence rules,
// kept on the device so that several updates run between read-backs.
// status codes: 0 = converged, 1 = running / not converged, 2 = diverged.
struct RecastState {
    double resid;     // relative change of the last update
    double first;     // norm of the first update's change
    double prev;      // norm of the previous update's change
    double dh[4];     // relative changes of the last four updates
    int status, iters, grow, pad;
};
constexpr int kRecastConverged = 0, kRecastRunning = 1, kRecastDiverged = 2;
// phi_new = scale * out / sa*, FP64 norms of the change; with st != nullptr
// the update also applies the loop's rules for update k (tolerance tol):
// a stopped instance's active flag is cleared, and a diverged one's field
// is zeroed.
void launch_recast_update(const float* out, const float* scale, float inv_sa_star, float* phi,
                          double* norms, int* active, RecastState* st, double tol, int k,
                          int B, int P, hipStream_t s);
// Per-instance resampling between a problem's grid (nf x nf, f = nf / nc)
// and the network grid (nc x nc).
struct ResampleDesc {
    const float *st, *ss, *q;   // the problem's fields
    float* guess;               // the problem's output field
    int nf, f;
};
void launch_recast_average(const ResampleDesc* d, int B, int nc, float* S, float* sa,
                           hipStream_t s);
void launch_recast_output(const ResampleDesc* d, int B, int nc, long long max_cells,
                          const float* phi, hipStream_t s);

// DeepONet helpers: g * (z > 0) elementwise, and column sums of an
// [R][C] row-major matrix in a fixed order (chunks of rows, then chunks in
// order; scratch holds ceil(R / kColChunk) * C floats).
constexpr int kColChunk = 128;
void launch_relu_back(const float* z, const float* g, float* out, long long n, hipStream_t s);
void launch_col_sum(const float* x, float* out, int R, int C, float* scratch, hipStream_t s);
void launch_grid_coords(float* xy, int n, hipStream_t s);

}  // namespace mdp
