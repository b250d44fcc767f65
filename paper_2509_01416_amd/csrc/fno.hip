// fno.hip -- kernels of the Fourier neural operator (arXiv 2509.01416
// section 4.2 and Appendix A1, in its 2-D form): a batched BF16 matrix-core
// GEMM with strided views that carries every dense contraction of the
// forward and backward passes (truncated DFTs as matrix products, pointwise
// 1x1 layers, projection), and the elementwise / reduction kernels around it
// (lift, GELU, per-mode complex mixing, projection head, bias and weight
// reductions, MSE, Adam).
//
// Activations are channel-major, [batch][channel][y][x] in FP32; GEMM
// operands are rounded to BF16 when staged into LDS and accumulated in FP32.
#include <math.h>

#include <type_traits>

#include "fno_kernels.h"

namespace mdp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned u = __builtin_bit_cast(unsigned, f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ long long vidx(int i, int ls, long long hi, long long lo) {
    return ls >= 31 ? (long long)i * lo
                    : (long long)(i >> ls) * hi + (long long)(i & ((1 << ls) - 1)) * lo;
}

__device__ __forceinline__ long long voff(const View& v, int g, int r, int c) {
    return vidx(g, v.b_ls, v.sb_hi, v.sb_lo) + vidx(r, v.r_ls, v.sr_hi, v.sr_lo) +
           vidx(c, v.c_ls, v.sc_hi, v.sc_lo);
}

// ------------------------------------------------------------------ GEMM --
// C[g] = alpha * A[g] (M x K) * B[g] (K x N) (+ C[g] if accumulate) (+ bias)
// 256 threads = 4 waves; a workgroup computes a 64 x 64 tile, each wave a
// 32 x 32 quadrant as 2 x 2 MFMA 16x16 tiles; K advances 32 per stage.
// BF16 operands use v_mfma_f32_16x16x16bf16_1k; the F32 instance (used to
// check the kernels against the FP64 oracle without BF16 rounding) uses
// v_mfma_f32_16x16x4f32.  With ksplit > 1, grid.z = G * ksplit and each
// slice writes its partial tile to `partial` [ksplit][G][M][N].
constexpr int kTile = 64, kTK = 32, kPad = 36;   // LDS row = 32 + 4 pad

template <bool F32>
__global__ void __launch_bounds__(256)
gemm_kernel(GemmArgs a) {
    typedef typename std::conditional<F32, float, unsigned short>::type T;
    __shared__ __attribute__((aligned(16))) T As[kTile * kPad];
    __shared__ __attribute__((aligned(16))) T Bs[kTile * kPad];   // transposed: Bs[n][k]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n0 = blockIdx.x * kTile, m0 = blockIdx.y * kTile;
    const int g = blockIdx.z / a.ksplit, kz = blockIdx.z - g * a.ksplit;
    const int kchunk = ((a.K + a.ksplit - 1) / a.ksplit + kTK - 1) / kTK * kTK;
    const int kbeg = kz * kchunk, kend = min(a.K, kbeg + kchunk);
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += kTK) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = tid + 256 * j;
            const int r = e >> 5, k = e & 31;          // A: row-major tile
            float va = 0.f;
            if (m0 + r < a.M && k0 + k < kend) va = a.A.p[voff(a.A, g, m0 + r, k0 + k)];
            const int kb = e >> 6, n = e & 63;         // B: k-major tile
            float vb = 0.f;
            if (n0 + n < a.N && k0 + kb < kend) vb = a.B.p[voff(a.B, g, k0 + kb, n0 + n)];
            if constexpr (F32) {
                As[r * kPad + k] = va;
                Bs[n * kPad + kb] = vb;
            } else {
                As[r * kPad + k] = to_bf16(va);
                Bs[n * kPad + kb] = to_bf16(vb);
            }
        }
        __syncthreads();
        if constexpr (F32) {
#pragma unroll
            for (int kk = 0; kk < kTK; kk += 4) {
                float af[2], bfr[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    af[t] = As[(wm + 16 * t + (lane & 15)) * kPad + kk + (lane >> 4)];
                    bfr[t] = Bs[(wn + 16 * t + (lane & 15)) * kPad + kk + (lane >> 4)];
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[j], acc[i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < kTK; kk += 16) {
                bf16x4 af[2], bfr[2];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    const T* pa = As + (wm + 16 * t + (lane & 15)) * kPad + kk + 4 * (lane >> 4);
                    const T* pb = Bs + (wn + 16 * t + (lane & 15)) * kPad + kk + 4 * (lane >> 4);
                    af[t] = *reinterpret_cast<const bf16x4*>(pa);
                    bfr[t] = *reinterpret_cast<const bf16x4*>(pb);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m >= a.M || n >= a.N) continue;
                const float v = acc[i][j][q];
                if (a.ksplit > 1) {
                    a.partial[(((long long)kz * a.G + g) * a.M + m) * a.N + n] = v;
                } else {
                    float* pc = a.C.p + voff(a.C, g, m, n);
                    float r = a.alpha * v;
                    if (a.accumulate) r += *pc;
                    if (a.bias_row) r += a.bias_row[m];
                    if (a.bias_col) r += a.bias_col[n];
                    *pc = r;
                }
            }
}

// Sum of split-K partials in slice order, then the epilogue.
__global__ void gemm_reduce_kernel(GemmArgs a) {
    const long long total = (long long)a.G * a.M * a.N;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(e % a.N);
        const int m = (int)((e / a.N) % a.M);
        const int g = (int)(e / ((long long)a.M * a.N));
        float s = 0.f;
        for (int kz = 0; kz < a.ksplit; ++kz) s += a.partial[(long long)kz * total + e];
        float* pc = a.C.p + voff(a.C, g, m, n);
        float r = a.alpha * s;
        if (a.accumulate) r += *pc;
        if (a.bias_row) r += a.bias_row[m];
        if (a.bias_col) r += a.bias_col[n];
        *pc = r;
    }
}

static long long hidx(int i, int ls, long long hi, long long lo) {
    return ls >= 31 ? (long long)i * lo : (long long)(i >> ls) * hi + (long long)(i & ((1 << ls) - 1)) * lo;
}

// Launches in chunks of batch entries so that grid.z stays below 65536; a
// chunk start must not split a batch view's low index range (checked).
bool launch_gemm(const GemmArgs& a0, hipStream_t s) {
    const int per = std::max(1, 65535 / a0.ksplit);
    for (int g0 = 0; g0 < a0.G; g0 += per) {
        GemmArgs a = a0;
        a.G = std::min(per, a0.G - g0);
        if (g0) {
            const View* vs[3] = {&a0.A, &a0.B, &a0.C};
            View* vd[3] = {&a.A, &a.B, &a.C};
            for (int t = 0; t < 3; ++t) {
                if (vs[t]->b_ls < 31 && (g0 & ((1 << vs[t]->b_ls) - 1))) return false;
                vd[t]->p = vs[t]->p + hidx(g0, vs[t]->b_ls, vs[t]->sb_hi, vs[t]->sb_lo);
            }
        }
        dim3 grid((a.N + kTile - 1) / kTile, (a.M + kTile - 1) / kTile, a.G * a.ksplit);
        if (a.f32)
            hipLaunchKernelGGL(gemm_kernel<true>, grid, dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL(gemm_kernel<false>, grid, dim3(256), 0, s, a);
        if (a.ksplit > 1) {
            const long long total = (long long)a.G * a.M * a.N;
            const int blocks = (int)std::min<long long>(4096, (total + 255) / 256);
            hipLaunchKernelGGL(gemm_reduce_kernel, dim3(blocks), dim3(256), 0, s, a);
        }
    }
    return true;
}

// --------------------------------------------------------------- helpers --
__device__ __forceinline__ float gelu_f(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Lift (input field, x/lx, y/ly) -> width channels.  in: [B][P];
// out: [B][C][P].  Cell-centre coordinates (i + 0.5)/n.
__global__ void lift_kernel(const float* __restrict__ in, const float* __restrict__ W0,
                            const float* __restrict__ b0, float* __restrict__ out,
                            int B, int n, int C) {
    const int P = n * n;
    const long long total = (long long)B * C * P;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(e % P);
        const int c = (int)((e / P) % C);
        const int b = (int)(e / ((long long)C * P));
        const float x = ((p % n) + 0.5f) / n, y = ((p / n) + 0.5f) / n;
        out[e] = fmaf(W0[c], in[(long long)b * P + p],
                      fmaf(W0[C + c], x, fmaf(W0[2 * C + c], y, b0[c])));
    }
}

__global__ void gelu_kernel(const float* __restrict__ z, float* __restrict__ v, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        v[e] = gelu_f(z[e]);
}

__global__ void gelu_back_kernel(const float* __restrict__ z, const float* __restrict__ gv,
                                 float* __restrict__ gz, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        gz[e] = gv[e] * gelu_grad_f(z[e]);
}

// Per-mode complex mixing.  X, Y: [B][C][2 (re,im)][2m (ky)][m (kx)];
// R: [2 blk][m][m][Ci][Co][2] (the flat parameter layout).
__global__ void mix_kernel(const float* __restrict__ X, const float* __restrict__ R,
                           float* __restrict__ Y, int B, int C, int m) {
    const int modes = 2 * m * m;
    const long long total = (long long)B * C * modes;
    const int per = 2 * 2 * m * m;   // floats per (b, c)
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int md = (int)(e % modes);
        const int o = (int)((e / modes) % C);
        const int b = (int)(e / ((long long)modes * C));
        const int kyi = md / m, kx = md - kyi * m;   // kyi in [0, 2m)
        const int blk = kyi / m, ky = kyi - blk * m;
        const float* w = R + ((((long long)blk * m + ky) * m + kx) * C) * C * 2;
        float yr = 0.f, yi = 0.f;
        for (int i = 0; i < C; ++i) {
            const float* xb = X + ((long long)b * C + i) * per;
            const float xr = xb[kyi * m + kx], xi = xb[2 * m * m + kyi * m + kx];
            const float wr = w[(i * C + o) * 2], wi = w[(i * C + o) * 2 + 1];
            yr = fmaf(xr, wr, fmaf(-xi, wi, yr));
            yi = fmaf(xr, wi, fmaf(xi, wr, yi));
        }
        float* yb = Y + ((long long)b * C + o) * per;
        yb[kyi * m + kx] = yr;
        yb[2 * m * m + kyi * m + kx] = yi;
    }
}

// gX[b][i] = sum_o gY[b][o] conj(R[i][o])
__global__ void mix_back_x_kernel(const float* __restrict__ gY, const float* __restrict__ R,
                                  float* __restrict__ gX, int B, int C, int m) {
    const int modes = 2 * m * m;
    const long long total = (long long)B * C * modes;
    const int per = 2 * 2 * m * m;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int md = (int)(e % modes);
        const int i = (int)((e / modes) % C);
        const int b = (int)(e / ((long long)modes * C));
        const int kyi = md / m, kx = md - kyi * m;
        const int blk = kyi / m, ky = kyi - blk * m;
        const float* w = R + ((((long long)blk * m + ky) * m + kx) * C) * C * 2;
        float gr = 0.f, gi = 0.f;
        for (int o = 0; o < C; ++o) {
            const float* gb = gY + ((long long)b * C + o) * per;
            const float yr = gb[kyi * m + kx], yi = gb[2 * m * m + kyi * m + kx];
            const float wr = w[(i * C + o) * 2], wi = w[(i * C + o) * 2 + 1];
            gr = fmaf(yr, wr, fmaf(yi, wi, gr));      // (yr + i yi)(wr - i wi)
            gi = fmaf(yi, wr, fmaf(-yr, wi, gi));
        }
        float* xb = gX + ((long long)b * C + i) * per;
        xb[kyi * m + kx] = gr;
        xb[2 * m * m + kyi * m + kx] = gi;
    }
}

// gR[i][o] = sum_b conj(X[b][i]) gY[b][o]  (batch order fixed)
__global__ void mix_back_w_kernel(const float* __restrict__ X, const float* __restrict__ gY,
                                  float* __restrict__ gR, int B, int C, int m) {
    const int modes = 2 * m * m;
    const long long total = (long long)modes * C * C;
    const int per = 2 * 2 * m * m;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int o = (int)(e % C);
        const int i = (int)((e / C) % C);
        const int md = (int)(e / ((long long)C * C));
        const int kyi = md / m, kx = md - kyi * m;
        const int blk = kyi / m, ky = kyi - blk * m;
        float gr = 0.f, gi = 0.f;
        for (int b = 0; b < B; ++b) {
            const float* xb = X + ((long long)b * C + i) * per;
            const float* yb = gY + ((long long)b * C + o) * per;
            const float xr = xb[kyi * m + kx], xi = xb[2 * m * m + kyi * m + kx];
            const float yr = yb[kyi * m + kx], yi = yb[2 * m * m + kyi * m + kx];
            gr = fmaf(xr, yr, fmaf(xi, yi, gr));      // (xr - i xi)(yr + i yi)
            gi = fmaf(xr, yi, fmaf(-xi, yr, gi));
        }
        float* w = gR + ((((long long)blk * m + ky) * m + kx) * C) * C * 2;
        w[(i * C + o) * 2] = gr;
        w[(i * C + o) * 2 + 1] = gi;
    }
}

// out[b][p] = sum_k P2[k] gelu(h[b][k][p]) + c2
__global__ void proj_out_kernel(const float* __restrict__ h, const float* __restrict__ P2,
                                const float* __restrict__ c2, float* __restrict__ out,
                                int B, int P, int K) {
    const long long total = (long long)B * P;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(e % P);
        const int b = (int)(e / P);
        const float* hb = h + (long long)b * K * P + p;
        float s = 0.f;
        for (int k = 0; k < K; ++k) s = fmaf(P2[k], gelu_f(hb[(long long)k * P]), s);
        out[e] = s + c2[0];
    }
}

// gh[b][k][p] = gout[b][p] P2[k] gelu'(h)
__global__ void proj_back_kernel(const float* __restrict__ h, const float* __restrict__ P2,
                                 const float* __restrict__ gout, float* __restrict__ gh,
                                 int B, int P, int K) {
    const long long total = (long long)B * K * P;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int p = (int)(e % P);
        const int k = (int)((e / P) % K);
        const int b = (int)(e / ((long long)K * P));
        gh[e] = gout[(long long)b * P + p] * P2[k] * gelu_grad_f(h[e]);
    }
}

// Row reductions with a fixed order: out[r] (+)= sum_{b, p} f(x[b][r][p]) y
// where the term is x (mode 0), x * w[b][p] (mode 1), or gelu(x) * w[b][p]
// (mode 2).  One block per row r; threads stride p, then a tree.
__global__ void row_reduce_kernel(const float* __restrict__ x, const float* __restrict__ w,
                                  float* __restrict__ out, int B, int Rr, int P, int mode,
                                  int accumulate) {
    const int r = blockIdx.x;
    float s = 0.f;
    for (int b = 0; b < B; ++b) {
        const float* xb = x + ((long long)b * Rr + r) * P;
        const float* wb = w ? w + (long long)b * P : nullptr;
        for (int p = threadIdx.x; p < P; p += blockDim.x) {
            float t = xb[p];
            if (mode == 2) t = gelu_f(t);
            if (mode >= 1) t *= wb[p];
            s += t;
        }
    }
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = (accumulate ? out[r] : 0.f) + red[0];
}

// Lift backward: gW0[j][c] = sum_{b,p} a_j gv0[b][c][p] (a_0 = input,
// a_1 = x, a_2 = y); gb0[c] = sum gv0.  One block per channel c.
__global__ void lift_back_kernel(const float* __restrict__ in, const float* __restrict__ gv,
                                 float* __restrict__ gW0, float* __restrict__ gb0,
                                 int B, int n, int C) {
    const int c = blockIdx.x;
    const int P = n * n;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int b = 0; b < B; ++b) {
        const float* g = gv + ((long long)b * C + c) * P;
        const float* a = in + (long long)b * P;
        for (int p = threadIdx.x; p < P; p += blockDim.x) {
            const float x = ((p % n) + 0.5f) / n, y = ((p / n) + 0.5f) / n;
            s0 = fmaf(a[p], g[p], s0);
            s1 = fmaf(x, g[p], s1);
            s2 = fmaf(y, g[p], s2);
            s3 += g[p];
        }
    }
    __shared__ float red[4][256];
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    red[3][threadIdx.x] = s3;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        gW0[c] = red[0][0];
        gW0[C + c] = red[1][0];
        gW0[2 * C + c] = red[2][0];
        gb0[c] = red[3][0];
    }
}

// MSE: per-block partial sums of (out - t)^2 and the gradient 2 (out - t)/n.
__global__ void mse_kernel(const float* __restrict__ out, const float* __restrict__ t,
                           float* __restrict__ gout, double* __restrict__ partial, long long n) {
    double s = 0.0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const float d = out[e] - t[e];
        s += (double)d * d;
        gout[e] = 2.0f * d / (float)n;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam (bias-corrected) on FP32 master parameters.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, long long n,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        const float mh = mm / c1, vh = vv / c2;
        p[e] -= lr * mh / (sqrtf(vh) + eps);
    }
}

// --------------------------------------------------------------- recast --
// One block per instance on the network grid: S_eff = S + (sa* - sa) phi,
// s = mean |S_eff|, in = S_eff / s.  Instances with active[b] == 0 are
// left untouched (their loop has already stopped).
__global__ void recast_input_kernel(const float* __restrict__ S, const float* __restrict__ sa,
                                    const float* __restrict__ phi, float sa_star,
                                    float* __restrict__ in, float* __restrict__ scale,
                                    const int* __restrict__ active, int P) {
    const int b = blockIdx.x;
    if (!active[b]) return;
    const float* Sb = S + (long long)b * P;
    const float* ab = sa + (long long)b * P;
    const float* pb = phi + (long long)b * P;
    float* ib = in + (long long)b * P;
    double s = 0.0;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        const float v = fmaf(sa_star - ab[p], pb[p], Sb[p]);
        ib[p] = v;
        s += fabs((double)v);
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const float sc = (float)(red[0] / P);
    if (threadIdx.x == 0) scale[b] = sc;
    const float inv = sc > 0.f ? 1.0f / sc : 0.f;
    for (int p = threadIdx.x; p < P; p += blockDim.x) ib[p] *= inv;
}

// phi_new = s * out / sa*; FP64 norms of the change and of phi_new.
__global__ void recast_update_kernel(const float* __restrict__ out, const float* __restrict__ scale,
                                     float inv_sa_star, float* __restrict__ phi,
                                     double* __restrict__ norms, const int* __restrict__ active,
                                     int P) {
    const int b = blockIdx.x;
    if (!active[b]) return;
    const float sc = scale[b] * inv_sa_star;
    double d2 = 0.0, n2 = 0.0;
    for (int p = threadIdx.x; p < P; p += blockDim.x) {
        const long long e = (long long)b * P + p;
        const float nv = out[e] * sc;
        const double d = (double)nv - (double)phi[e];
        d2 += d * d;
        n2 += (double)nv * nv;
        phi[e] = nv;
    }
    __shared__ double r1[256], r2[256];
    r1[threadIdx.x] = d2;
    r2[threadIdx.x] = n2;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            r1[threadIdx.x] += r1[threadIdx.x + h];
            r2[threadIdx.x] += r2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        norms[2 * b] = r1[0];
        norms[2 * b + 1] = r2[0];
    }
}

// Block average of a fine field (f x f blocks) onto the network grid.
__global__ void block_average_kernel(const float* __restrict__ fine, int nf_x, int f,
                                     float* __restrict__ coarse, int nc, const float* __restrict__ sub,
                                     int mode) {
    const int P = nc * nc;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < P; e += gridDim.x * blockDim.x) {
        const int X = e % nc, Y = e / nc;
        double s = 0.0;
        for (int j = 0; j < f; ++j)
            for (int i = 0; i < f; ++i) {
                const long long c = (long long)(Y * f + j) * nf_x + (X * f + i);
                s += mode == 0 ? (double)fine[c] : (double)fine[c] - (double)sub[c];
            }
        coarse[e] = (float)(s / (f * f));
    }
}

// Bilinear interpolation (cell-centred, edges clamped) of a coarse field to
// a fine grid that is an integer multiple f of it.
__global__ void bilinear_up_kernel(const float* __restrict__ coarse, int nc, int f,
                                   float* __restrict__ fine, float scale) {
    const int nf = nc * f;
    const long long P = (long long)nf * nf;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < P;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e % nf), j = (int)(e / nf);
        const float xc = (i + 0.5f) / f - 0.5f, yc = (j + 0.5f) / f - 0.5f;
        int i0 = (int)floorf(xc), j0 = (int)floorf(yc);
        float tx = xc - i0, ty = yc - j0;
        int i1 = i0 + 1, j1 = j0 + 1;
        if (i0 < 0) { i0 = 0; tx = 0.f; }
        if (j0 < 0) { j0 = 0; ty = 0.f; }
        if (i1 > nc - 1) { i1 = nc - 1; }
        if (j1 > nc - 1) { j1 = nc - 1; }
        if (i0 > nc - 1) { i0 = nc - 1; }
        if (j0 > nc - 1) { j0 = nc - 1; }
        const float v00 = coarse[j0 * nc + i0], v10 = coarse[j0 * nc + i1];
        const float v01 = coarse[j1 * nc + i0], v11 = coarse[j1 * nc + i1];
        const float a = v00 + tx * (v10 - v00), b = v01 + tx * (v11 - v01);
        fine[e] = scale * (a + ty * (b - a));
    }
}

__global__ void scale_kernel(float* __restrict__ x, float s, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        x[e] *= s;
}

// ------------------------------------------------------------- launchers --
static int blocks_for(long long n) {
    return (int)std::max<long long>(1, std::min<long long>(8192, (n + 255) / 256));
}

void launch_lift(const float* in, const float* W0, const float* b0, float* out, int B,
                 int n, int C, hipStream_t s) {
    const long long t = (long long)B * C * n * n;
    hipLaunchKernelGGL(lift_kernel, dim3(blocks_for(t)), dim3(256), 0, s, in, W0, b0, out, B, n, C);
}
void launch_gelu(const float* z, float* v, long long n, hipStream_t s) {
    hipLaunchKernelGGL(gelu_kernel, dim3(blocks_for(n)), dim3(256), 0, s, z, v, n);
}
void launch_gelu_back(const float* z, const float* gv, float* gz, long long n, hipStream_t s) {
    hipLaunchKernelGGL(gelu_back_kernel, dim3(blocks_for(n)), dim3(256), 0, s, z, gv, gz, n);
}
void launch_mix(const float* X, const float* R, float* Y, int B, int C, int m, hipStream_t s) {
    const long long t = (long long)B * C * 2 * m * m;
    hipLaunchKernelGGL(mix_kernel, dim3(blocks_for(t)), dim3(256), 0, s, X, R, Y, B, C, m);
}
void launch_mix_back_x(const float* gY, const float* R, float* gX, int B, int C, int m,
                       hipStream_t s) {
    const long long t = (long long)B * C * 2 * m * m;
    hipLaunchKernelGGL(mix_back_x_kernel, dim3(blocks_for(t)), dim3(256), 0, s, gY, R, gX, B, C, m);
}
void launch_mix_back_w(const float* X, const float* gY, float* gR, int B, int C, int m,
                       hipStream_t s) {
    const long long t = (long long)2 * m * m * C * C;
    hipLaunchKernelGGL(mix_back_w_kernel, dim3(blocks_for(t)), dim3(256), 0, s, X, gY, gR, B, C, m);
}
void launch_proj_out(const float* h, const float* P2, const float* c2, float* out, int B,
                     int P, int K, hipStream_t s) {
    hipLaunchKernelGGL(proj_out_kernel, dim3(blocks_for((long long)B * P)), dim3(256), 0, s, h,
                       P2, c2, out, B, P, K);
}
void launch_proj_back(const float* h, const float* P2, const float* gout, float* gh, int B,
                      int P, int K, hipStream_t s) {
    hipLaunchKernelGGL(proj_back_kernel, dim3(blocks_for((long long)B * K * P)), dim3(256), 0,
                       s, h, P2, gout, gh, B, P, K);
}
void launch_row_reduce(const float* x, const float* w, float* out, int B, int R, int P,
                       int mode, int accumulate, hipStream_t s) {
    hipLaunchKernelGGL(row_reduce_kernel, dim3(R), dim3(256), 0, s, x, w, out, B, R, P, mode,
                       accumulate);
}
void launch_lift_back(const float* in, const float* gv, float* gW0, float* gb0, int B, int n,
                      int C, hipStream_t s) {
    hipLaunchKernelGGL(lift_back_kernel, dim3(C), dim3(256), 0, s, in, gv, gW0, gb0, B, n, C);
}
int launch_mse(const float* out, const float* t, float* gout, double* partial, long long n,
               hipStream_t s) {
    const int blocks = (int)std::min<long long>(256, (n + 255) / 256);
    hipLaunchKernelGGL(mse_kernel, dim3(blocks), dim3(256), 0, s, out, t, gout, partial, n);
    return blocks;
}
void launch_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1,
                       b2, eps, c1, c2);
}
void launch_recast_input(const float* S, const float* sa, const float* phi, float sa_star,
                         float* in, float* scale, const int* active, int B, int P,
                         hipStream_t s) {
    hipLaunchKernelGGL(recast_input_kernel, dim3(B), dim3(256), 0, s, S, sa, phi, sa_star, in,
                       scale, active, P);
}
void launch_recast_update(const float* out, const float* scale, float inv_sa_star, float* phi,
                          double* norms, const int* active, int B, int P, hipStream_t s) {
    hipLaunchKernelGGL(recast_update_kernel, dim3(B), dim3(256), 0, s, out, scale, inv_sa_star,
                       phi, norms, active, P);
}
void launch_block_average(const float* fine, int nf_x, int f, float* coarse, int nc,
                          const float* sub, int mode, hipStream_t s) {
    hipLaunchKernelGGL(block_average_kernel, dim3(blocks_for((long long)nc * nc)), dim3(256), 0,
                       s, fine, nf_x, f, coarse, nc, sub, mode);
}
void launch_bilinear_up(const float* coarse, int nc, int f, float* fine, float scale,
                        hipStream_t s) {
    const long long P = (long long)nc * f * nc * f;
    hipLaunchKernelGGL(bilinear_up_kernel, dim3(blocks_for(P)), dim3(256), 0, s, coarse, nc, f,
                       fine, scale);
}
void launch_scale(float* x, float sc, long long n, hipStream_t s) {
    hipLaunchKernelGGL(scale_kernel, dim3(blocks_for(n)), dim3(256), 0, s, x, sc, n);
}

}  // namespace mdp
