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

// Round to nearest even (gfx950's conversion instruction).
__device__ __forceinline__ unsigned short to_bf16(float f) {
    return __builtin_bit_cast(unsigned short, (__bf16)f);
}

__device__ __forceinline__ float gelu_dev(float z) {
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

// GELU for the BF16-operand path, with erfc from the rational approximation
// of Abramowitz & Stegun 7.1.26 (Hastings): for a >= 0,
//   erfc(a) ~= t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-a^2),
//   t = 1 / (1 + p a),  |error| <= 1.5e-7,
// so gelu(z) = z (1 + erf(z / sqrt 2)) / 2 = (z + |z| (1 - erfc(|z| / sqrt 2))) / 2
// to within 1e-7 |z|: about half the instructions of erff, far below the
// BF16 rounding of the operands it feeds.  The FP32 checking mode keeps erff.
__device__ __forceinline__ float gelu_fast(float z) {
    const float h = 0.5f * fabsf(z);
    const float a = h * 1.41421356237309505f;                 // |z| / sqrt 2
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, a, 1.0f));
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    q = q * t * __builtin_amdgcn_exp2f(a * (a * -1.44269504088896341f));   // erfc(a)
    return fmaf(-h, q, h) + 0.5f * z;
}

template <bool F32>
__device__ __forceinline__ float gelu_op(float z) {
    if constexpr (F32) return gelu_dev(z);
    else return gelu_fast(z);
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
//
// Staging: each thread stages 8 elements of A and 8 of B per K-stage.  The
// thread-to-element map walks the operand's unit-stride axis with
// consecutive threads (coalesced), and one view offset is computed per
// stage; the other 7 elements follow at a constant stride (a split index
// never breaks inside a 64-row tile or a 32-wide K stage, since splits are
// at multiples of 64).
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
    // A map: k-fast (unit stride along K): m = (tid >> 5) + 8 j, k = tid & 31;
    //        m-fast: m = tid & 63, k = (tid >> 6) + 4 j.
    const bool a_kfast = a.A.sc_lo == 1 && a.A.c_ls >= 5;
    const int am = a_kfast ? (tid >> 5) : (tid & 63);
    const int ak = a_kfast ? (tid & 31) : (tid >> 6);
    const long long astep = a_kfast ? 8 * a.A.sr_lo : 4 * a.A.sc_lo;
    // B map: n-fast: k = (tid >> 6) + 4 j, n = tid & 63;
    //        k-fast: k = tid & 31, n = (tid >> 5) + 8 j.
    const bool b_nfast = a.B.sc_lo == 1 && a.B.c_ls >= 6;
    const int bk = b_nfast ? (tid >> 6) : (tid & 31);
    const int bn = b_nfast ? (tid & 63) : (tid >> 5);
    const long long bstep = b_nfast ? 4 * a.B.sr_lo : 8 * a.B.sc_lo;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // The global values of stage k0 + kTK are loaded into registers while
    // the matrix cores work on stage k0.  Every load is unconditional (an
    // element outside the operand reads the view's first element instead and
    // is replaced by zero), so the 16 loads of a thread go out together.
    float ra[8], rb[8];
    auto load_stage = [&](int k0) {
        const int kk = k0 + ak;
        const float* pa = a.A.p + voff(a.A, g, m0 + am, kk);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int m = a_kfast ? am + 8 * j : am;
            const int k = a_kfast ? ak : ak + 4 * j;
            const bool in = m0 + m < a.M && k0 + k < kend;
            const float v = *(in ? pa + j * astep : a.A.p);
            ra[j] = in ? v : 0.f;
        }
        const float* pb = a.B.p + voff(a.B, g, k0 + bk, n0 + bn);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = b_nfast ? bk + 4 * j : bk;
            const int n = b_nfast ? bn : bn + 8 * j;
            const bool in = n0 + n < a.N && k0 + k < kend;
            const float v = *(in ? pb + j * bstep : a.B.p);
            rb[j] = in ? v : 0.f;
        }
    };
    if (kbeg < kend) load_stage(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += kTK) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int m = a_kfast ? am + 8 * j : am;
            const int k = a_kfast ? ak : ak + 4 * j;
            if constexpr (F32) As[m * kPad + k] = ra[j];
            else As[m * kPad + k] = to_bf16(ra[j]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = b_nfast ? bk + 4 * j : bk;
            const int n = b_nfast ? bn : bn + 8 * j;
            if constexpr (F32) Bs[n * kPad + k] = rb[j];
            else Bs[n * kPad + k] = to_bf16(rb[j]);
        }
        __syncthreads();
        if (k0 + kTK < kend) load_stage(k0 + kTK);
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
                    const long long oc = voff(a.C, g, m, n);
                    float r = a.alpha * v;
                    if (a.accumulate) r += a.C.p[oc];
                    if (a.bias_row) r += a.bias_row[m];
                    if (a.bias_col) r += a.bias_col[n];
                    a.C.p[oc] = r;
                    if (a.gelu_out) a.gelu_out[oc] = gelu_dev(r);
                    if (a.relu_out) a.relu_out[oc] = fmaxf(r, 0.f);
                }
            }
}

// Sum of split-K partials in slice order, then the epilogue.
// Fixed-order split-K reduction: a workgroup takes 64 consecutive outputs
// (coalesced partial loads) and kRedWaves waves; wave w sums the slices
// kz = w, w + kRedWaves, ... in order, and the wave sums are added in wave
// order before the epilogue.
constexpr int kRedWaves = 16;
__global__ void __launch_bounds__(64 * kRedWaves) gemm_reduce_kernel(GemmArgs a) {
    const long long total = (long long)a.G * a.M * a.N;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long e = (long long)blockIdx.x * 64 + lane;
    __shared__ float ps[kRedWaves][64];
    float s = 0.f;
    if (e < total) {
#pragma unroll 4
        for (int kz = w; kz < a.ksplit; kz += kRedWaves) s += a.partial[(long long)kz * total + e];
    }
    ps[w][lane] = s;
    __syncthreads();
    if (w != 0 || e >= total) return;
    float t = 0.f;
#pragma unroll
    for (int v = 0; v < kRedWaves; ++v) t += ps[v][lane];
    const int n = (int)(e % a.N);
    const int m = (int)((e / a.N) % a.M);
    const int g = (int)(e / ((long long)a.M * a.N));
    float* pc = a.C.p + voff(a.C, g, m, n);
    float r = a.alpha * t;
    if (a.accumulate) r += *pc;
    if (a.bias_row) r += a.bias_row[m];
    if (a.bias_col) r += a.bias_col[n];
    *pc = r;
    if (a.gelu_out) a.gelu_out[pc - a.C.p] = gelu_dev(r);
    if (a.relu_out) a.relu_out[pc - a.C.p] = fmaxf(r, 0.f);
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
            hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((total + 63) / 64)),
                               dim3(64 * kRedWaves), 0, s, a);
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
    // grid (ceil(n*n / 256), B): one pixel per thread, all C channels (the
    // input is read once; each channel's stores are coalesced)
    const int P = n * n;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (p >= P) return;
    const int iy = p / n, ix = p - iy * n;
    const float x = (ix + 0.5f) / n, y = (iy + 0.5f) / n;
    const float v = in[(size_t)b * P + p];
    float* ob = out + (size_t)b * C * P + p;
    for (int c = 0; c < C; ++c)
        ob[(size_t)c * P] = fmaf(W0[c], v, fmaf(W0[C + c], x, fmaf(W0[2 * C + c], y, b0[c])));
}

__global__ void gelu_back_kernel(const float* __restrict__ z, const float* __restrict__ gv,
                                 float* __restrict__ gz, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        gz[e] = gv[e] * gelu_grad_f(z[e]);
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

// Two-stage row reductions with a fixed order.  Stage 1: block (r, chunk)
// sums 1024 consecutive cells of sample chunk/nsub of row r (threads stride
// the cells, then a tree) into part[r * nchunk + chunk]; stage 2 sums a
// row's chunks in chunk order.  Term: x (mode 0), x w (1), gelu(x) w (2).
constexpr int kRedCells = 1024;

__global__ void __launch_bounds__(256)
row_reduce_part_kernel(const float* __restrict__ x, const float* __restrict__ w,
                       float* __restrict__ part, int Rr, int P, int mode) {
    const int r = blockIdx.x, ch = blockIdx.y, nch = gridDim.y;
    const int nsub = P / kRedCells;
    const int b = ch / nsub, p0 = (ch - b * nsub) * kRedCells;
    const float* xb = x + ((long long)b * Rr + r) * P + p0;
    const float* wb = w ? w + (long long)b * P + p0 : nullptr;
    float s = 0.f;
    for (int p = threadIdx.x; p < kRedCells; p += blockDim.x) {
        float t = xb[p];
        if (mode == 2) t = gelu_f(t);
        if (mode >= 1) t *= wb[p];
        s += t;
    }
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long long)r * nch + ch] = red[0];
}

__global__ void row_reduce_fin_kernel(const float* __restrict__ part, float* __restrict__ out,
                                      int Rr, int nch, int accumulate) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= Rr) return;
    float s = 0.f;
    for (int c = 0; c < nch; ++c) s += part[(long long)r * nch + c];
    out[r] = (accumulate ? out[r] : 0.f) + s;
}

// Lift backward in two stages: block (c, chunk) forms the four sums
// (input, x, y, 1) x gv0 over 1024 cells; stage 2 sums chunks in order.
__global__ void __launch_bounds__(256)
lift_back_part_kernel(const float* __restrict__ in, const float* __restrict__ gv,
                      float* __restrict__ part, int n, int C) {
    const int c = blockIdx.x, ch = blockIdx.y, nch = gridDim.y;
    const int P = n * n, nsub = P / kRedCells;
    const int b = ch / nsub, p0 = (ch - b * nsub) * kRedCells;
    const float* g = gv + ((long long)b * C + c) * P;
    const float* a = in + (long long)b * P;
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int p = p0 + threadIdx.x; p < p0 + kRedCells; p += blockDim.x) {
        const float x = ((p % n) + 0.5f) / n, y = ((p / n) + 0.5f) / n;
        s0 = fmaf(a[p], g[p], s0);
        s1 = fmaf(x, g[p], s1);
        s2 = fmaf(y, g[p], s2);
        s3 += g[p];
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
    if (threadIdx.x < 4) part[((long long)threadIdx.x * C + c) * nch + ch] = red[threadIdx.x][0];
}

__global__ void lift_back_fin_kernel(const float* __restrict__ part, float* __restrict__ gW0,
                                     float* __restrict__ gb0, int C, int nch) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;   // q * C + c
    if (e >= 4 * C) return;
    const int q = e / C, c = e - q * C;
    float s = 0.f;
    for (int k = 0; k < nch; ++k) s += part[(long long)e * nch + k];
    if (q < 3) gW0[q * C + c] = s;
    else gb0[c] = s;
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
    // 64 x 64 grid with 16-byte aligned rows: each thread keeps its 16 cells
    // in registers (four float4 loads per field issued together)
    constexpr int kR = 4;
    const bool regs = P == kR * 4 * 256 && blockDim.x == 256 &&
                      ((reinterpret_cast<size_t>(Sb) | reinterpret_cast<size_t>(ab) |
                        reinterpret_cast<size_t>(pb) | reinterpret_cast<size_t>(ib)) & 15) == 0;
    float4 v4[kR];
    if (regs) {
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const int e = (k * 256 + (int)threadIdx.x) * 4;
            const float4 S4 = *reinterpret_cast<const float4*>(Sb + e);
            const float4 a4 = *reinterpret_cast<const float4*>(ab + e);
            const float4 p4 = *reinterpret_cast<const float4*>(pb + e);
            v4[k] = make_float4(fmaf(sa_star - a4.x, p4.x, S4.x), fmaf(sa_star - a4.y, p4.y, S4.y),
                                fmaf(sa_star - a4.z, p4.z, S4.z), fmaf(sa_star - a4.w, p4.w, S4.w));
        }
#pragma unroll
        for (int k = 0; k < kR; ++k)
            s += fabs((double)v4[k].x) + fabs((double)v4[k].y) + fabs((double)v4[k].z) +
                 fabs((double)v4[k].w);
    } else {
        for (int p = threadIdx.x; p < P; p += blockDim.x) {
            const float v = fmaf(sa_star - ab[p], pb[p], Sb[p]);
            ib[p] = v;
            s += fabs((double)v);
        }
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
    if (regs) {
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const int e = (k * 256 + (int)threadIdx.x) * 4;
            *reinterpret_cast<float4*>(ib + e) =
                make_float4(v4[k].x * inv, v4[k].y * inv, v4[k].z * inv, v4[k].w * inv);
        }
    } else {
        for (int p = threadIdx.x; p < P; p += blockDim.x) ib[p] *= inv;
    }
}

// The recast loop's rules for one instance after update k, from the FP64
// squared norms of the change (d2) and of the new field (n2): converged when
// the relative change d falls below tol, or when it has stalled close to it
// (d < 10 tol and less than 10 % below the change three updates earlier:
// the network's rounding floor); diverged when the change is not finite, or
// its norm has grown three updates in a row to above the first update's.
// Returns true when the instance diverged.
__device__ bool recast_rules(RecastState& s, double d2, double n2, double tol, int k,
                             int* active) {
    const double num = sqrt(d2), den = sqrt(n2);
    const double d = den > 0.0 ? num / den : (num == 0.0 ? 0.0 : INFINITY);
    s.iters = k + 1;
    s.resid = d;
    int done = -1;
    s.dh[k & 3] = d;
    if (!isfinite(d) || !isfinite(num)) {
        done = kRecastDiverged;
    } else if (d < tol) {
        done = kRecastConverged;
    } else if (k >= 3 && d < 10.0 * tol && d > 0.9 * s.dh[(k - 3) & 3]) {
        done = kRecastConverged;
    } else {
        s.grow = (k >= 1 && num > s.prev) ? s.grow + 1 : 0;
        if (k == 0) s.first = num;
        if (s.grow >= 3 && num > s.first) done = kRecastDiverged;
    }
    s.prev = num;
    if (done >= 0) {
        s.status = done;
        *active = 0;
    }
    return done == kRecastDiverged;
}

// phi_new = s * out / sa*; FP64 norms of the change and of phi_new; with a
// state array, the loop's rules for update k (a diverged instance's field is
// zeroed: the fallback is the zero start).
__global__ void recast_update_kernel(const float* __restrict__ out, const float* __restrict__ scale,
                                     float inv_sa_star, float* __restrict__ phi,
                                     double* __restrict__ norms, int* __restrict__ active,
                                     RecastState* __restrict__ st, double tol, int k, int P) {
    const int b = blockIdx.x;
    if (!active[b]) return;
    const float sc = scale[b] * inv_sa_star;
    double d2 = 0.0, n2 = 0.0;
    const float* ob = out + (long long)b * P;
    float* fb = phi + (long long)b * P;
    constexpr int kR = 4;
    if (P == kR * 4 * 256 && blockDim.x == 256 &&
        ((reinterpret_cast<size_t>(ob) | reinterpret_cast<size_t>(fb)) & 15) == 0) {
        // 64 x 64 grid: all loads of a thread issued together
        float4 o4[kR], f4[kR];
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const int e = (k * 256 + (int)threadIdx.x) * 4;
            o4[k] = *reinterpret_cast<const float4*>(ob + e);
            f4[k] = *reinterpret_cast<const float4*>(fb + e);
        }
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const float nv[4] = {o4[k].x * sc, o4[k].y * sc, o4[k].z * sc, o4[k].w * sc};
            const float ov[4] = {f4[k].x, f4[k].y, f4[k].z, f4[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double d = (double)nv[j] - (double)ov[j];
                d2 += d * d;
                n2 += (double)nv[j] * nv[j];
            }
            *reinterpret_cast<float4*>(fb + (k * 256 + (int)threadIdx.x) * 4) =
                make_float4(nv[0], nv[1], nv[2], nv[3]);
        }
    } else {
        for (int p = threadIdx.x; p < P; p += blockDim.x) {
            const float nv = ob[p] * sc;
            const double d = (double)nv - (double)fb[p];
            d2 += d * d;
            n2 += (double)nv * nv;
            fb[p] = nv;
        }
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
    __shared__ int zero_phi;
    if (threadIdx.x == 0) {
        norms[2 * b] = r1[0];
        norms[2 * b + 1] = r2[0];
        zero_phi = st != nullptr && recast_rules(st[b], r1[0], r2[0], tol, k, active + b);
    }
    __syncthreads();
    if (zero_phi)
        for (int p = threadIdx.x; p < P; p += blockDim.x) fb[p] = 0.f;
}

// Block averages of every instance's fields onto the network grid (f x f
// blocks, FP64 sums in row order): S = mean(q), sa = mean(sigma_t -
// sigma_s).  Grid (ceil(nc*nc / 256), instances).
__global__ void recast_average_kernel(const ResampleDesc* __restrict__ d, int nc,
                                      float* __restrict__ S, float* __restrict__ sa) {
    const int b = blockIdx.y;
    const int P = nc * nc;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P) return;
    const ResampleDesc r = d[b];
    const int X = e % nc, Y = e / nc, f = r.f;
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j < f; ++j)
        for (int i = 0; i < f; ++i) {
            const long long c = (long long)(Y * f + j) * r.nf + (X * f + i);
            s1 += (double)r.q[c];
            s2 += (double)r.st[c] - (double)r.ss[c];
        }
    S[(long long)b * P + e] = (float)(s1 / (f * f));
    sa[(long long)b * P + e] = (float)(s2 / (f * f));
}

// Every instance's guess on its own grid: a copy when f = 1, else
// cell-centred bilinear interpolation with clamped edges.  Grid
// (ceil(max fine cells / 256), instances).
__global__ void recast_output_kernel(const ResampleDesc* __restrict__ d, int nc,
                                     const float* __restrict__ phi) {
    const int b = blockIdx.y;
    const ResampleDesc r = d[b];
    const int f = r.f, nf = r.nf;
    const long long P = (long long)nf * nf;
    const float* coarse = phi + (long long)b * nc * nc;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < P;
         e += (long long)gridDim.x * blockDim.x) {
        if (f == 1) {
            r.guess[e] = coarse[e];
            continue;
        }
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
        const float a = v00 + tx * (v10 - v00), bb = v01 + tx * (v11 - v01);
        r.guess[e] = a + ty * (bb - a);
    }
}

// ------------------------------------------------------- per-mode mixing --
// One workgroup per retained mode (kyi, kx): that mode's weights
// R[i][o] (32 x 32 complex, contiguous in the parameter vector) and the
// batch's mode values are staged in LDS; the batch is processed in chunks of
// kMixChunk samples.  X, Y: [B][C][2 (re,im)][2m (ky)][m (kx)];
// R: [2 blk][m][m][Ci][Co][2] (the flat parameter layout).
constexpr int kMixChunk = 64;

__global__ void __launch_bounds__(256)
mix_mode_kernel(const float* __restrict__ X, const float* __restrict__ R,
                float* __restrict__ Y, int B, int C, int m) {
    extern __shared__ float sm[];
    float* Rs = sm;                         // [C][C][2]
    float* Xs = sm + 2 * C * C;             // [chunk][C][2]
    const int md = blockIdx.x;              // kyi * m + kx
    const int kyi = md / m, kx = md - kyi * m;
    const int blk = kyi / m, ky = kyi - blk * m;
    const int per = 4 * m * m, plane = 2 * m * m;
    const float* w = R + ((((long long)blk * m + ky) * m + kx) * C) * C * 2;
    for (int e = threadIdx.x; e < 2 * C * C; e += blockDim.x) Rs[e] = w[e];
    for (int b0 = 0; b0 < B; b0 += kMixChunk) {
        const int nb = min(kMixChunk, B - b0);
        __syncthreads();
        for (int e = threadIdx.x; e < nb * C; e += blockDim.x) {
            const float* xb = X + ((long long)(b0 * C) + e) * per;
            Xs[2 * e] = xb[md];
            Xs[2 * e + 1] = xb[plane + md];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nb * C; e += blockDim.x) {
            const int b = e / C, o = e - b * C;
            const float* xr = Xs + 2 * b * C;
            float yr = 0.f, yi = 0.f;
            for (int i = 0; i < C; ++i) {
                const float xre = xr[2 * i], xim = xr[2 * i + 1];
                const float wr = Rs[(i * C + o) * 2], wi = Rs[(i * C + o) * 2 + 1];
                yr = fmaf(xre, wr, fmaf(-xim, wi, yr));
                yi = fmaf(xre, wi, fmaf(xim, wr, yi));
            }
            float* yb = Y + ((long long)(b0 * C) + e) * per;
            yb[md] = yr;
            yb[plane + md] = yi;
        }
    }
}

// gX[b][i] = sum_o gY[b][o] conj(R[i][o])
__global__ void __launch_bounds__(256)
mix_mode_back_x_kernel(const float* __restrict__ gY, const float* __restrict__ R,
                       float* __restrict__ gX, int B, int C, int m) {
    extern __shared__ float sm[];
    float* Rs = sm;
    float* Gs = sm + 2 * C * C;
    const int md = blockIdx.x;
    const int kyi = md / m, kx = md - kyi * m;
    const int blk = kyi / m, ky = kyi - blk * m;
    const int per = 4 * m * m, plane = 2 * m * m;
    const float* w = R + ((((long long)blk * m + ky) * m + kx) * C) * C * 2;
    // transposed, Rs[o][i], so that threads with consecutive i read
    // consecutive LDS words
    for (int e = threadIdx.x; e < C * C; e += blockDim.x) {
        const int i = e / C, o = e - i * C;
        Rs[(o * C + i) * 2] = w[2 * e];
        Rs[(o * C + i) * 2 + 1] = w[2 * e + 1];
    }
    for (int b0 = 0; b0 < B; b0 += kMixChunk) {
        const int nb = min(kMixChunk, B - b0);
        __syncthreads();
        for (int e = threadIdx.x; e < nb * C; e += blockDim.x) {
            const float* gb = gY + ((long long)(b0 * C) + e) * per;
            Gs[2 * e] = gb[md];
            Gs[2 * e + 1] = gb[plane + md];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nb * C; e += blockDim.x) {
            const int b = e / C, i = e - b * C;
            const float* gr = Gs + 2 * b * C;
            float xr = 0.f, xi = 0.f;
            for (int o = 0; o < C; ++o) {
                const float yr = gr[2 * o], yi = gr[2 * o + 1];
                const float wr = Rs[(o * C + i) * 2], wi = Rs[(o * C + i) * 2 + 1];
                xr = fmaf(yr, wr, fmaf(yi, wi, xr));
                xi = fmaf(yi, wr, fmaf(-yr, wi, xi));
            }
            float* xb = gX + ((long long)(b0 * C) + e) * per;
            xb[md] = xr;
            xb[plane + md] = xi;
        }
    }
}

// gR[i][o] = sum_b conj(X[b][i]) gY[b][o], batch order fixed
__global__ void __launch_bounds__(256)
mix_mode_back_w_kernel(const float* __restrict__ X, const float* __restrict__ gY,
                       float* __restrict__ gR, int B, int C, int m) {
    extern __shared__ float sm[];
    float* Xs = sm;                         // [chunk][C][2]
    float* Gs = sm + 2 * kMixChunk * C;     // [chunk][C][2]
    const int md = blockIdx.x;
    const int kyi = md / m, kx = md - kyi * m;
    const int blk = kyi / m, ky = kyi - blk * m;
    const int per = 4 * m * m, plane = 2 * m * m;
    float accr[4] = {0.f, 0.f, 0.f, 0.f}, acci[4] = {0.f, 0.f, 0.f, 0.f};
    const int nout = C * C;
    for (int b0 = 0; b0 < B; b0 += kMixChunk) {
        const int nb = min(kMixChunk, B - b0);
        __syncthreads();
        for (int e = threadIdx.x; e < nb * C; e += blockDim.x) {
            const long long src = ((long long)(b0 * C) + e) * per;
            Xs[2 * e] = X[src + md];
            Xs[2 * e + 1] = X[src + plane + md];
            Gs[2 * e] = gY[src + md];
            Gs[2 * e + 1] = gY[src + plane + md];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + q * blockDim.x;
            if (e >= nout) break;
            const int i = e / C, o = e - i * C;
            float gr = accr[q], gi = acci[q];
            for (int b = 0; b < nb; ++b) {
                const float xr = Xs[2 * (b * C + i)], xi = Xs[2 * (b * C + i) + 1];
                const float yr = Gs[2 * (b * C + o)], yi = Gs[2 * (b * C + o) + 1];
                gr = fmaf(xr, yr, fmaf(xi, yi, gr));
                gi = fmaf(xr, yi, fmaf(-xi, yr, gi));
            }
            accr[q] = gr;
            acci[q] = gi;
        }
    }
    float* w = gR + ((((long long)blk * m + ky) * m + kx) * C) * C * 2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = threadIdx.x + q * blockDim.x;
        if (e >= nout) break;
        w[2 * e] = accr[q];
        w[2 * e + 1] = acci[q];
    }
}

// ------------------------------------------------- fused projection head --
// out[b][p] = c2 + sum_k P2[k] gelu(h[b][k][p]),  h = P1^T v + c1 (K = 128
// hidden units, C = 32 input channels).  One workgroup per (64-pixel tile,
// sample): wave w computes hidden units 32w..32w+31 for the 64 pixels with
// 2 x 4 MFMA tiles, applies c1, GELU and P2, reduces its 32 rows, and the
// four waves' sums are added in wave order.  h is also stored when h_out is
// given (training needs it).  P (pixels per sample) is a multiple of 4.
template <bool F32>
__global__ void __launch_bounds__(256)
proj_fused_kernel(const float* __restrict__ v, const float* __restrict__ P1,
                  const float* __restrict__ c1, const float* __restrict__ P2,
                  const float* __restrict__ c2, float* __restrict__ out,
                  float* __restrict__ h_out, int P) {
    typedef typename std::conditional<F32, float, unsigned short>::type T;
    constexpr int C = 32, K = 128, NT = 64;
    __shared__ __attribute__((aligned(16))) T Ws[K * (C + 4)];    // P1^T [k][c]
    __shared__ __attribute__((aligned(16))) T Vs[NT * (C + 4)];   // [pixel][c]
    __shared__ float part[4][NT];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int p0 = blockIdx.x * NT, b = blockIdx.y;
    const float* vb = v + (long long)b * C * P;
    const int km = wv * 32;
    // every global load of the thread first (P % 4 == 0): P1 (four float4),
    // the tile of v (two float4), and the c1 / P2 entries of its epilogue
    float4 pr[K * C / 4 / 256], vr[C * NT / 4 / 256];
#pragma unroll
    for (int i = 0; i < K * C / 4 / 256; ++i)
        pr[i] = reinterpret_cast<const float4*>(P1)[tid + 256 * i];
#pragma unroll
    for (int i = 0; i < C * NT / 4 / 256; ++i) {
        const int e4 = tid + 256 * i, c = e4 / (NT / 4), pp = 4 * (e4 % (NT / 4));
        const bool in = p0 + pp < P;
        vr[i] = *reinterpret_cast<const float4*>(vb + (long long)c * P + (in ? p0 + pp : 0));
        if (!in) vr[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float ck[2][4], pk[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = km + 16 * i + 4 * (lane >> 4) + q;
            ck[i][q] = c1[k];
            pk[i][q] = P2[k];
        }
#pragma unroll
    for (int i = 0; i < K * C / 4 / 256; ++i) {          // P1[c][k] -> Ws[k][c]
        const int e = 4 * (tid + 256 * i), c = e / K, k = e - c * K;
        const float x[4] = {pr[i].x, pr[i].y, pr[i].z, pr[i].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (F32) Ws[(k + j) * (C + 4) + c] = x[j];
            else Ws[(k + j) * (C + 4) + c] = to_bf16(x[j]);
        }
    }
#pragma unroll
    for (int i = 0; i < C * NT / 4 / 256; ++i) {         // v[c][p] -> Vs[p][c]
        const int e4 = tid + 256 * i, c = e4 / (NT / 4), pp = 4 * (e4 % (NT / 4));
        const float x[4] = {vr[i].x, vr[i].y, vr[i].z, vr[i].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (F32) Vs[(pp + j) * (C + 4) + c] = x[j];
            else Vs[(pp + j) * (C + 4) + c] = to_bf16(x[j]);
        }
    }
    __syncthreads();
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (F32) {
#pragma unroll
        for (int kk = 0; kk < C; kk += 4) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const float af = Ws[(km + 16 * i + (lane & 15)) * (C + 4) + kk + (lane >> 4)];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float bf = Vs[(16 * j + (lane & 15)) * (C + 4) + kk + (lane >> 4)];
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf, acc[i][j], 0, 0, 0);
                }
            }
        }
    } else {
#pragma unroll
        for (int kk = 0; kk < C; kk += 16) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const bf16x4 af = *reinterpret_cast<const bf16x4*>(
                    Ws + (km + 16 * i + (lane & 15)) * (C + 4) + kk + 4 * (lane >> 4));
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bf16x4 bf = *reinterpret_cast<const bf16x4*>(
                        Vs + (16 * j + (lane & 15)) * (C + 4) + kk + 4 * (lane >> 4));
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf, acc[i][j], 0, 0, 0);
                }
            }
        }
    }
    // lane holds rows km + 16i + 4(lane>>4) + q, column 16j + (lane & 15)
    float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = km + 16 * i + 4 * (lane >> 4) + q;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float hv = acc[i][j][q] + ck[i][q];
                const int pp = 16 * j + (lane & 15);
                if (h_out && p0 + pp < P) h_out[((long long)b * K + k) * P + p0 + pp] = hv;
                s[j] = fmaf(pk[i][q], gelu_op<F32>(hv), s[j]);
            }
        }
    // reduce over the four row groups of the wave (lanes l, l+16, l+32, l+48)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float t = s[j];
        t += __shfl_xor(t, 16, 64);
        t += __shfl_xor(t, 32, 64);
        s[j] = t;
    }
    if (lane < 16)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[wv][16 * j + lane] = s[j];
    __syncthreads();
    if (tid < NT && p0 + tid < P) {
        const float r = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
        out[(long long)b * P + p0 + tid] = r + c2[0];
    }
}

// ------------------------------------------------ fused spectral kernels --
// One workgroup (4 waves) per (sample, channel) of a 64 x 64 field with the
// retained-mode window of 12 x (12 + 12) modes.  Operands are staged in LDS
// (BF16, or FP32 for the checking mode) in the layouts the MFMA fragments
// read: A as [m][k], B as [n][k] (k contiguous).
//   spec_fwd:  T (64 x 24) = V (64 x 64) . FxT (64 x 24);  X (48 x 12) = Fy (48 x 128) . [T_re; T_im]
//   spec_inv:  Z (128 x 12) = Gy (128 x 48) . Y (48 x 12); U (64 x 64) = Z' (64 x 24) . Gx (24 x 64)
// The products accumulate in FP32 in the same k order as the batched GEMM.
template <bool F32>
struct Frag;
template <>
struct Frag<false> {
    typedef unsigned short T;
    static constexpr int KS = 16;   // k per MFMA
    __device__ static T cvt(float x) { return to_bf16(x); }
    __device__ static f32x4 mma(const T* a, const T* b, int lane, f32x4 c) {
        const bf16x4 af = *reinterpret_cast<const bf16x4*>(a + 4 * (lane >> 4));
        const bf16x4 bf = *reinterpret_cast<const bf16x4*>(b + 4 * (lane >> 4));
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af, bf, c, 0, 0, 0);
    }
};
template <>
struct Frag<true> {
    typedef float T;
    static constexpr int KS = 4;
    __device__ static T cvt(float x) { return x; }
    __device__ static f32x4 mma(const T* a, const T* b, int lane, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a[lane >> 4], b[lane >> 4], c, 0, 0, 0);
    }
};

// C tile (16 x 16) at (m0, n0) of A [m][lda] . B^T [n][ldb] over k in [0, K).
template <bool F32>
__device__ __forceinline__ f32x4 tile_mma(const typename Frag<F32>::T* A, int lda,
                                          const typename Frag<F32>::T* Bt, int ldb, int m0,
                                          int n0, int K, int lane) {
    f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f};
    const typename Frag<F32>::T* a = A + (m0 + (lane & 15)) * lda;
    const typename Frag<F32>::T* b = Bt + (n0 + (lane & 15)) * ldb;
    for (int k = 0; k < K; k += Frag<F32>::KS) c = Frag<F32>::mma(a + k, b + k, lane, c);
    return c;
}

// LDS images of the DFT matrices, built once per model (stage_spec_kernel):
// the exact padded layouts the two kernels below keep in LDS, per operand
// precision, so a workgroup copies them with 16-byte loads.
constexpr int kSpLV = 64 + 8, kSpLT = 128 + 8, kSpLG = 48 + 8, kSpLZ = 32 + 8;
constexpr int kImgFx = 0;                          // [32][LV]  FxT^T, rows >= 24 zero
constexpr int kImgFy = kImgFx + 32 * kSpLV;        // [48][LT]  Fy
constexpr int kImgGy = kImgFy + 48 * kSpLT;        // [128][LG] Gy
constexpr int kImgGx = kImgGy + 128 * kSpLG;       // [64][LZ]  Gx^T, columns >= 24 zero
constexpr int kImgElems = kImgGx + 64 * kSpLZ;     // elements per precision

template <bool F32>
__global__ void stage_spec_kernel(const float* __restrict__ FxT, const float* __restrict__ Fy,
                                  const float* __restrict__ Gy, const float* __restrict__ Gx,
                                  typename Frag<F32>::T* __restrict__ img) {
    constexpr int n = 64, mm = 12;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kImgElems; e += gridDim.x * blockDim.x) {
        float v = 0.f;
        if (e < kImgFy) {
            const int j = e / kSpLV, x = e % kSpLV;
            if (j < 2 * mm && x < n) v = FxT[x * 2 * mm + j];
        } else if (e < kImgGy) {
            const int r = (e - kImgFy) / kSpLT, k = (e - kImgFy) % kSpLT;
            if (k < 2 * n) v = Fy[r * 2 * n + k];
        } else if (e < kImgGx) {
            const int r = (e - kImgGy) / kSpLG, k = (e - kImgGy) % kSpLG;
            if (k < 4 * mm) v = Gy[r * 4 * mm + k];
        } else {
            const int x = (e - kImgGx) / kSpLZ, k = (e - kImgGx) % kSpLZ;
            if (k < 2 * mm) v = Gx[k * n + x];
        }
        img[e] = Frag<F32>::cvt(v);
    }
}

// 16-byte copy of `bytes` (a multiple of 16) from global to LDS by 256 threads
// Global -> LDS copy of BYTES (a multiple of 16) by 256 threads: all loads
// of a thread are issued before its stores (a thread past the end reloads
// the last chunk and stores nothing).
template <int BYTES>
__device__ __forceinline__ void copy16(void* dst, const void* src) {
    static_assert(BYTES % 16 == 0, "16-byte chunks");
    constexpr int N = BYTES / 16, IT = (N + 255) / 256;
    const uint4* s = reinterpret_cast<const uint4*>(src);
    uint4* d = reinterpret_cast<uint4*>(dst);
    uint4 r[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) r[i] = s[min((int)threadIdx.x + 256 * i, N - 1)];
#pragma unroll
    for (int i = 0; i < IT; ++i)
        if ((int)threadIdx.x + 256 * i < N) d[threadIdx.x + 256 * i] = r[i];
}

// 64 x 64 FP32 field -> registers (four float4 per thread), then -> LDS
// [y][LV] in the operand precision
__device__ __forceinline__ void load_field(float4 (&r)[4], const float* vg) {
    const float4* v4 = reinterpret_cast<const float4*>(vg);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = v4[threadIdx.x + 256 * k];
}
template <bool F32>
__device__ __forceinline__ void store_field(typename Frag<F32>::T* Vs, const float4 (&r)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = threadIdx.x + 256 * k;        // float4 index: y = e / 16
        const float4 v = r[k];
        typename Frag<F32>::T* d = Vs + (e >> 4) * kSpLV + 4 * (e & 15);
        if constexpr (F32) {
            *reinterpret_cast<float4*>(d) = v;
        } else {
            const unsigned lo = (unsigned)to_bf16(v.x) | ((unsigned)to_bf16(v.y) << 16);
            const unsigned hi = (unsigned)to_bf16(v.z) | ((unsigned)to_bf16(v.w) << 16);
            *reinterpret_cast<uint2*>(d) = make_uint2(lo, hi);
        }
    }
}

template <bool F32>
__device__ __forceinline__ void zero_lds(typename Frag<F32>::T* p, int elems) {
    uint4* d = reinterpret_cast<uint4*>(p);
    const int n16 = elems * (int)sizeof(typename Frag<F32>::T) / 16;
    for (int e = threadIdx.x; e < n16; e += 256) d[e] = make_uint4(0u, 0u, 0u, 0u);
}

// One lifted value (LiftArgs): channel c, input u at cell (ix, iy) of the
// 64 x 64 grid, with lift_kernel's arithmetic.
__device__ __forceinline__ float lift_value(const LiftArgs& L, int c, float u, int ix, int iy) {
    constexpr int C = 32, n = 64;
    const float x = (ix + 0.5f) / n, y = (iy + 0.5f) / n;
    return fmaf(L.W0[c], u, fmaf(L.W0[C + c], x, fmaf(L.W0[2 * C + c], y, L.b0[c])));
}

// A workgroup transforms CH consecutive fields: the DFT images are staged
// once, and the next field's values are loaded while the current one is on
// the matrix cores.  With lift.in the fields are the lift of the network
// input, formed here (32 channels).
template <bool F32, int CH>
__global__ void __launch_bounds__(256)
spec_fwd_kernel(const float* __restrict__ v, const typename Frag<F32>::T* __restrict__ img,
                float* __restrict__ X, int G, LiftArgs lift) {
    typedef typename Frag<F32>::T T;
    constexpr int n = 64, mm = 12, LV = kSpLV, LT = kSpLT;
    __shared__ __attribute__((aligned(16))) T Vs[n * LV];          // [y][x]
    __shared__ __attribute__((aligned(16))) T Fx[32 * LV];         // [j][x], j < 24 used
    __shared__ __attribute__((aligned(16))) T Fys[48 * LT];        // [(q,kyi)][(p,y)]
    __shared__ __attribute__((aligned(16))) T Ts[16 * LT];         // [kx][(p,y)]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long long g0 = (long long)blockIdx.x * CH;
    float4 fr[4];
    auto load_v = [&](long long g) {
        if (lift.in == nullptr) {
            load_field(fr, v + g * n * n);
            return;
        }
        const int c = (int)(g % 32);
        const float4* in4 = reinterpret_cast<const float4*>(lift.in + (g / 32) * n * n);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = threadIdx.x + 256 * k, iy = e >> 4, ix = 4 * (e & 15);
            const float4 u = in4[e];
            fr[k] = make_float4(lift_value(lift, c, u.x, ix, iy),
                                lift_value(lift, c, u.y, ix + 1, iy),
                                lift_value(lift, c, u.z, ix + 2, iy),
                                lift_value(lift, c, u.w, ix + 3, iy));
        }
    };
    load_v(g0);
    copy16<32 * LV * (int)sizeof(T)>(Fx, img + kImgFx);
    copy16<48 * LT * (int)sizeof(T)>(Fys, img + kImgFy);
    zero_lds<F32>(Ts, 16 * LT);   // rows kx >= 12 stay zero
    for (int ci = 0; ci < CH; ++ci) {
        const long long g = g0 + ci;
        if (g >= G) break;
        store_field<F32>(Vs, fr);
        __syncthreads();
        if (ci + 1 < CH && g + 1 < G) load_v(g + 1);
        // T: wave w owns rows 16w..16w+15, both 16-column tiles
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const f32x4 c = tile_mma<F32>(Vs, LV, Fx, LV, 16 * wv, 16 * t, n, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int y = 16 * wv + 4 * (lane >> 4) + q, j = 16 * t + (lane & 15);
                if (j < 2 * mm) Ts[(j % mm) * LT + (j / mm) * n + y] = Frag<F32>::cvt(c[q]);
            }
        }
        __syncthreads();
        // X: waves 0..2 own rows 16w..16w+15 (48 rows), one 16-column tile
        if (wv < 3) {
            const f32x4 c = tile_mma<F32>(Fys, LT, Ts, LT, 16 * wv, 0, 128, lane);
            float* xg = X + g * 48 * mm;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * wv + 4 * (lane >> 4) + q, kx = lane & 15;
                if (kx < mm) xg[r * mm + kx] = c[q];
            }
        }
    }
}

template <bool F32, int CH>
__global__ void __launch_bounds__(256)
spec_inv_kernel(const float* __restrict__ Y, const typename Frag<F32>::T* __restrict__ img,
                float* __restrict__ U, int G) {
    typedef typename Frag<F32>::T T;
    constexpr int n = 64, mm = 12, LG = kSpLG, LZ = kSpLZ;
    __shared__ __attribute__((aligned(16))) T Gys[128 * LG];       // [(p,y)][(q,kyi)]
    __shared__ __attribute__((aligned(16))) T Ys[16 * LG];         // [kx][(q,kyi)]
    __shared__ __attribute__((aligned(16))) T Zs[n * LZ];          // [y][(p,kx)], 24 of 32 used
    __shared__ __attribute__((aligned(16))) T Gxs[n * LZ];         // [x][(p,kx)]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const long long g0 = (long long)blockIdx.x * CH;
    // Y[r][kx] -> Ys[kx][r]: three entries per thread (e = tid + 256 i,
    // kx = e / 48 < 16); entries with kx >= 12 are zero
    float yr[3];
    auto load_y = [&](long long g) {
        const float* yg = Y + g * 48 * mm;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int e = tid + 256 * i, kx = e / 48, r = e % 48;
            yr[i] = yg[r * mm + min(kx, mm - 1)];
            if (kx >= mm) yr[i] = 0.f;
        }
    };
    load_y(g0);
    copy16<128 * LG * (int)sizeof(T)>(Gys, img + kImgGy);
    copy16<n * LZ * (int)sizeof(T)>(Gxs, img + kImgGx);
    zero_lds<F32>(Zs, n * LZ);    // columns (p,kx) >= 24 stay zero
    for (int ci = 0; ci < CH; ++ci) {
        const long long g = g0 + ci;
        if (g >= G) break;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int e = tid + 256 * i, kx = e / 48, r = e % 48;
            Ys[kx * LG + r] = Frag<F32>::cvt(yr[i]);
        }
        __syncthreads();
        if (ci + 1 < CH && g + 1 < G) load_y(g + 1);
        // Z: wave w owns rows 32w..32w+31 (two 16-row tiles), one column tile
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int m0 = 32 * wv + 16 * t;
            const f32x4 c = tile_mma<F32>(Gys, LG, Ys, LG, m0, 0, 48, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = m0 + 4 * (lane >> 4) + q, kx = lane & 15;   // r = p*64 + y
                if (kx < mm) Zs[(r & 63) * LZ + (r >> 6) * mm + kx] = Frag<F32>::cvt(c[q]);
            }
        }
        __syncthreads();
        // U: wave w owns rows 16w..16w+15, four column tiles
        float* ug = U + g * n * n;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const f32x4 c = tile_mma<F32>(Zs, LZ, Gxs, LZ, 16 * wv, 16 * t, 32, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int y = 16 * wv + 4 * (lane >> 4) + q, x = 16 * t + (lane & 15);
                ug[y * n + x] = c[q];
            }
        }
    }
}

// ------------------------------------------------- per-mode mixing (MMA) --
// For every retained mode, Y[b][:] = X[b][:] R (32 x 32 complex), written as
// one real product on the matrix cores in FP32:
//   [Yr | Yi] (16 x 64) = [Xr | Xi] (16 x 64) . [[Rr, Ri], [-Ri, Rr]] (64 x 64)
// X, Y: [B][32][2][2m][m] (modes contiguous); R: [2m][m][Ci][Co][2].
// Four consecutive modes per workgroup, one per wave, and one tile of 16
// batch rows (zero-padded) per workgroup row of the grid.  X is read and Y
// written as float4 over the four modes.
constexpr int kMixLA = 64 + 4;
// Rr / Ri row pitch: 16 mod 32 words, so the two half-waves of a fragment
// read (k rows k, k + 1 and k + 2, k + 3) each hit 32 distinct banks
constexpr int kMixLR = 48;
__global__ void __launch_bounds__(256)
mix_mma_kernel(const float* __restrict__ X, const float* __restrict__ R,
               float* __restrict__ Y, int B, int plane) {
    constexpr int C = 32, LA = kMixLA, LR = kMixLR;
    // As: [mode][b][k]; Rs: [mode][part][ci][co] (row pitch LR), which after
    // the products holds Os: [b][n][mode]
    __shared__ __attribute__((aligned(16))) float As[4 * 16 * LA];
    __shared__ __attribute__((aligned(16))) float Rs[4 * 2 * C * LR];
    float* Os = Rs;
    static_assert(16 * 64 * 4 <= 4 * 2 * C * LR, "output staging fits the weight buffer");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int md0 = 4 * blockIdx.x, per = 2 * plane;
    const int b0 = 16 * blockIdx.y;
    // all global loads of a thread first: 8 x two complex weights (the four
    // modes' 2048 complex weights each), 4 x four modes of X
    float4 wr[4 * C * C / 2 / 256], xr[16 * C * 2 / 256];
#pragma unroll
    for (int i = 0; i < 4 * C * C / 2 / 256; ++i) {
        const int e = tid + 256 * i;
        const int j = e >> 9, cc = (e & 511) * 2;
        wr[i] = *reinterpret_cast<const float4*>(R + (size_t)(md0 + j) * C * C * 2 + 2 * cc);
    }
#pragma unroll
    for (int i = 0; i < 16 * C * 2 / 256; ++i) {          // (b, c, part)
        const int e = tid + 256 * i;
        const int bb = e >> 6, c = (e >> 1) & 31, part = e & 1;
        const int bs = min(b0 + bb, B - 1);                 // rows past B load row B-1
        xr[i] = *reinterpret_cast<const float4*>(X + ((size_t)bs * C + c) * per + part * plane +
                                                 md0);
        if (b0 + bb >= B) xr[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < 4 * C * C / 2 / 256; ++i) {
        const int e = tid + 256 * i;
        const int j = e >> 9, cc = (e & 511) * 2;            // two complex weights
        const int ci = cc >> 5, co = cc & 31;
        float* Rj = Rs + j * 2 * C * LR;
        Rj[ci * LR + co] = wr[i].x;
        Rj[(C + ci) * LR + co] = wr[i].y;
        Rj[ci * LR + co + 1] = wr[i].z;
        Rj[(C + ci) * LR + co + 1] = wr[i].w;
    }
#pragma unroll
    for (int i = 0; i < 16 * C * 2 / 256; ++i) {
        const int e = tid + 256 * i;
        const int bb = e >> 6, c = (e >> 1) & 31, part = e & 1;
        const float4 x = xr[i];
        const int k = part * 32 + c;
        As[(0 * 16 + bb) * LA + k] = x.x;
        As[(1 * 16 + bb) * LA + k] = x.y;
        As[(2 * 16 + bb) * LA + k] = x.z;
        As[(3 * 16 + bb) * LA + k] = x.w;
    }
    __syncthreads();
    // wave wv: mode md0 + wv; output column tiles n0 = 16 t of the 64 x 64
    // real operand B[n][k] = [[Rr, Ri], [-Ri, Rr]] (n = part_out * 32 + co,
    // k = part_in * 32 + ci), read from the compact Rr / Ri planes with the
    // k order of the other matrix-core products
    f32x4 acc[4];
    {
        const float* Aw = As + wv * 16 * LA + (lane & 15) * LA + (lane >> 4);
        const float* Rw = Rs + wv * 2 * C * LR;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2 * C; kk += 4) {
                const bool im = (t >= 2) != (kk >= C);           // Ri block
                const float* rb = Rw + ((im ? C : 0) + (kk & (C - 1)) + (lane >> 4)) * LR +
                                  16 * (t & 1) + (lane & 15);
                const float bv = (t < 2 && kk >= C) ? -*rb : *rb;
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(Aw[kk], bv, acc[t], 0, 0, 0);
            }
        }
    }
    __syncthreads();   // every wave is done with Rs
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            Os[((4 * (lane >> 4) + q) * 64 + 16 * t + (lane & 15)) * 4 + wv] = acc[t][q];
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += 256) {               // (b, n = part * 32 + co)
        const int bb = e >> 6, n = e & 63;
        if (b0 + bb < B)
            *reinterpret_cast<float4*>(Y + ((size_t)(b0 + bb) * C + (n & 31)) * per +
                                       (n >> 5) * plane + md0) =
                *reinterpret_cast<const float4*>(Os + e * 4);
    }
}

// ------------------------------------------------- pointwise layer path --
// z[b][co][p] += sum_ci W[ci][co] v[b][ci][p] + bias[co] (z holds the
// spectral path on entry); optionally gelu(z) into vn.  C = 32 channels.
// One workgroup per (64-pixel tile, sample): wave w computes output rows
// 16 (w & 1) .. +15 and pixels 32 (w >> 1) .. +31 as two 16 x 16 MFMA tiles,
// with the batched GEMM's operand rounding and k order (so the results are
// those of the strided GEMM for this shape).  store_z = 0 leaves z as it is
// (inference: the next layer reads only gelu(z)).  With lift.in, v is the
// lift of the network input, formed here.
template <bool F32>
__global__ void __launch_bounds__(256)
pointwise_kernel(const float* __restrict__ W, const float* __restrict__ v,
                 const float* __restrict__ bias, float* __restrict__ z,
                 float* __restrict__ vn, int P, int store_z, LiftArgs lift) {
    typedef typename Frag<F32>::T T;
    constexpr int C = 32, LK = C + 4;
    __shared__ __attribute__((aligned(16))) T As[C * LK];    // [co][ci]
    __shared__ __attribute__((aligned(16))) T Bs[64 * LK];   // [p][ci]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int p0 = blockIdx.x * 64, b = blockIdx.y;
    const size_t base = (size_t)b * C * P;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = tid + 256 * k;                          // W[ci][co], e = ci * 32 + co
        As[(e & 31) * LK + (e >> 5)] = Frag<F32>::cvt(W[e]);
    }
    {
        const int ci = tid >> 3, n0 = (tid & 7) * 8;           // 8 pixels of channel ci
        const float4* src =
            lift.in == nullptr
                ? reinterpret_cast<const float4*>(v + base + (size_t)ci * P + p0 + n0)
                : reinterpret_cast<const float4*>(lift.in + (size_t)b * P + p0 + n0);
        const float4 x0 = src[0], x1 = src[1];
        float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        if (lift.in != nullptr) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int p = p0 + n0 + j;
                xs[j] = lift_value(lift, ci, xs[j], p & 63, p >> 6);
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) Bs[(n0 + j) * LK + ci] = Frag<F32>::cvt(xs[j]);
    }
    __syncthreads();
    const int m0 = 16 * (wv & 1);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int n0 = 32 * (wv >> 1) + 16 * t;
        const f32x4 c = tile_mma<F32>(As, LK, Bs, LK, m0, n0, C, lane);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int m = m0 + 4 * (lane >> 4) + q, p = p0 + n0 + (lane & 15);
            const size_t o = base + (size_t)m * P + p;
            float r = c[q];
            r += z[o];
            r += bias[m];
            if (store_z) z[o] = r;
            if (vn) vn[o] = gelu_op<F32>(r);
        }
    }
}

// ----------------------------- last pointwise layer + projection head --
// The last Fourier layer's pointwise path fused with the projection head,
// for 32 channels and 128 hidden units.  One workgroup per (64-pixel tile,
// sample), the tiling both kernels use: z = W^T v + (spectral path) + bias
// for the tile's 32 channels with pointwise_kernel's products, rounding and
// order; z goes to LDS as the head's operand, rounded as proj_fused_kernel
// rounds the z it reads; then proj_fused_kernel's products, GELU and
// fixed-order sums: out = c2 + sum_k P2[k] gelu(P1^T z + c1)[k].  The
// results are the two kernels' bit for bit.  z (on entry the spectral
// path) is stored when store_z (a backward pass reads it), h when h_out.
template <bool F32>
__global__ void __launch_bounds__(256)
pointwise_proj_kernel(const float* __restrict__ W, const float* __restrict__ v,
                      const float* __restrict__ bias, float* __restrict__ z, int store_z,
                      const float* __restrict__ P1, const float* __restrict__ c1,
                      const float* __restrict__ P2, const float* __restrict__ c2,
                      float* __restrict__ out, float* __restrict__ h_out, int P) {
    typedef typename Frag<F32>::T T;
    constexpr int C = 32, K = 128, NT = 64, LK = C + 4;
    __shared__ __attribute__((aligned(16))) T As[C * LK];     // W^T [co][ci]
    __shared__ __attribute__((aligned(16))) T Bs[NT * LK];    // v [pixel][ci]
    __shared__ __attribute__((aligned(16))) T Ws[K * LK];     // P1^T [k][c]
    __shared__ __attribute__((aligned(16))) T Vs[NT * LK];    // z [pixel][c]
    __shared__ float part[4][NT];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int p0 = blockIdx.x * NT, b = blockIdx.y;
    const size_t base = (size_t)b * C * P;
    const int km = wv * 32;
    // global loads first: P1 (four float4), the v tile (two float4), W, and
    // the c1 / P2 entries of the head's epilogue
    float4 pr[K * C / 4 / 256];
#pragma unroll
    for (int i = 0; i < K * C / 4 / 256; ++i)
        pr[i] = reinterpret_cast<const float4*>(P1)[tid + 256 * i];
    const int vci = tid >> 3, vn0 = (tid & 7) * 8;            // 8 pixels of channel vci
    const float4* vsrc = reinterpret_cast<const float4*>(v + base + (size_t)vci * P + p0 + vn0);
    const float4 x0 = vsrc[0], x1 = vsrc[1];
    float wr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) wr[k] = W[tid + 256 * k];
    float ck[2][4], pk[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = km + 16 * i + 4 * (lane >> 4) + q;
            ck[i][q] = c1[k];
            pk[i][q] = P2[k];
        }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int e = tid + 256 * k;                          // W[ci][co], e = ci * 32 + co
        As[(e & 31) * LK + (e >> 5)] = Frag<F32>::cvt(wr[k]);
    }
    {
        const float xs[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) Bs[(vn0 + j) * LK + vci] = Frag<F32>::cvt(xs[j]);
    }
#pragma unroll
    for (int i = 0; i < K * C / 4 / 256; ++i) {           // P1[c][k] -> Ws[k][c]
        const int e = 4 * (tid + 256 * i), c = e / K, k = e - c * K;
        const float x[4] = {pr[i].x, pr[i].y, pr[i].z, pr[i].w};
#pragma unroll
        for (int j = 0; j < 4; ++j) Ws[(k + j) * LK + c] = Frag<F32>::cvt(x[j]);
    }
    __syncthreads();
    // pointwise path: wave w, output rows 16 (w & 1) .. +15, pixels
    // 32 (w >> 1) .. +31 as two 16 x 16 tiles
    {
        const int m0 = 16 * (wv & 1);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int n0 = 32 * (wv >> 1) + 16 * t;
            const f32x4 c = tile_mma<F32>(As, LK, Bs, LK, m0, n0, C, lane);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + 4 * (lane >> 4) + q, pp = n0 + (lane & 15);
                const size_t o = base + (size_t)m * P + p0 + pp;
                float r = c[q];
                r += z[o];
                r += bias[m];
                if (store_z) z[o] = r;
                Vs[pp * LK + m] = Frag<F32>::cvt(r);
            }
        }
    }
    __syncthreads();
    // projection head: wave w, hidden units 32w .. 32w+31 for the 64 pixels
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < C; kk += Frag<F32>::KS) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const T* a = Ws + (km + 16 * i + (lane & 15)) * LK + kk;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T* bp = Vs + (16 * j + (lane & 15)) * LK + kk;
                acc[i][j] = Frag<F32>::mma(a, bp, lane, acc[i][j]);
            }
        }
    }
    // lane holds rows km + 16i + 4(lane>>4) + q, column 16j + (lane & 15)
    float sm[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = km + 16 * i + 4 * (lane >> 4) + q;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float hv = acc[i][j][q] + ck[i][q];
                const int pp = 16 * j + (lane & 15);
                if (h_out) h_out[((long long)b * K + k) * P + p0 + pp] = hv;
                sm[j] = fmaf(pk[i][q], gelu_op<F32>(hv), sm[j]);
            }
        }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float t = sm[j];
        t += __shfl_xor(t, 16, 64);
        t += __shfl_xor(t, 32, 64);
        sm[j] = t;
    }
    if (lane < 16)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[wv][16 * j + lane] = sm[j];
    __syncthreads();
    if (tid < NT) {
        const float r = ((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid];
        out[(long long)b * P + p0 + tid] = r + c2[0];
    }
}

// ------------------------------------------------------------- launchers --
static int blocks_for(long long n) {
    return (int)std::max<long long>(1, std::min<long long>(8192, (n + 255) / 256));
}

void launch_lift(const float* in, const float* W0, const float* b0, float* out, int B,
                 int n, int C, hipStream_t s) {
    for (int b0i = 0; b0i < B; b0i += 65535) {   // grid.z limit
        const int nb = std::min(65535, B - b0i);
        const size_t P = (size_t)n * n;
        hipLaunchKernelGGL(lift_kernel, dim3((n * n + 255) / 256, nb), dim3(256), 0, s,
                           in + b0i * P, W0, b0, out + b0i * P * C, nb, n, C);
    }
}
void launch_gelu_back(const float* z, const float* gv, float* gz, long long n, hipStream_t s) {
    hipLaunchKernelGGL(gelu_back_kernel, dim3(blocks_for(n)), dim3(256), 0, s, z, gv, gz, n);
}
void launch_mix(const float* X, const float* R, float* Y, int B, int C, int m, hipStream_t s) {
    if (C == 32 && (2 * m * m) % 4 == 0) {
        hipLaunchKernelGGL(mix_mma_kernel, dim3(2 * m * m / 4, (B + 15) / 16), dim3(256), 0, s, X, R, Y, B,
                           2 * m * m);
        return;
    }
    const size_t lds = sizeof(float) * (2 * C * C + 2 * kMixChunk * C);
    hipLaunchKernelGGL(mix_mode_kernel, dim3(2 * m * m), dim3(256), lds, s, X, R, Y, B, C, m);
}
void launch_mix_back_x(const float* gY, const float* R, float* gX, int B, int C, int m,
                       hipStream_t s) {
    const size_t lds = sizeof(float) * (2 * C * C + 2 * kMixChunk * C);
    hipLaunchKernelGGL(mix_mode_back_x_kernel, dim3(2 * m * m), dim3(256), lds, s, gY, R, gX,
                       B, C, m);
}
void launch_mix_back_w(const float* X, const float* gY, float* gR, int B, int C, int m,
                       hipStream_t s) {
    const size_t lds = sizeof(float) * (4 * kMixChunk * C);
    hipLaunchKernelGGL(mix_mode_back_w_kernel, dim3(2 * m * m), dim3(256), lds, s, X, gY, gR,
                       B, C, m);
}
size_t spec_image_bytes() {
    return (size_t)kImgElems * (sizeof(float) + sizeof(unsigned short));
}
// img: [FP32 image][BF16 image]
void launch_stage_spec(const float* FxT, const float* Fy, const float* Gy, const float* Gx,
                       void* img, hipStream_t s) {
    float* f = reinterpret_cast<float*>(img);
    unsigned short* h = reinterpret_cast<unsigned short*>(f + kImgElems);
    hipLaunchKernelGGL(stage_spec_kernel<true>, dim3(64), dim3(256), 0, s, FxT, Fy, Gy, Gx, f);
    hipLaunchKernelGGL(stage_spec_kernel<false>, dim3(64), dim3(256), 0, s, FxT, Fy, Gy, Gx, h);
}
void launch_pointwise(const float* W, const float* v, const float* bias, float* z, float* vn,
                      int B, int P, int store_z, int f32, hipStream_t s, const LiftArgs& lift) {
    dim3 grid(P / 64, B);
    if (f32)
        hipLaunchKernelGGL(pointwise_kernel<true>, grid, dim3(256), 0, s, W, v, bias, z, vn, P,
                           store_z, lift);
    else
        hipLaunchKernelGGL(pointwise_kernel<false>, grid, dim3(256), 0, s, W, v, bias, z, vn, P,
                           store_z, lift);
}
// fields per workgroup: the most (up to 8) that still leave two workgroups
// per CU (at batch 64 that is 7 % faster per forward than one per CU; at
// batch 16 and below no different)
static int spec_fields_per_wg(int G) {
    int ch = 8;
    while (ch > 1 && (G + ch - 1) / ch < 512) ch >>= 1;
    return ch;
}
#define MDP_SPEC_LAUNCH(kern)                                                              \
    template <bool F32>                                                                    \
    static void launch_##kern(const float* in, const typename Frag<F32>::T* img, float* o,  \
                              int G, hipStream_t s) {                                      \
        const int ch = spec_fields_per_wg(G);                                             \
        const dim3 grid((unsigned)((G + ch - 1) / ch));                                    \
        switch (ch) {                                                                      \
            case 8: hipLaunchKernelGGL((kern<F32, 8>), grid, dim3(256), 0, s, in, img, o, G); break; \
            case 4: hipLaunchKernelGGL((kern<F32, 4>), grid, dim3(256), 0, s, in, img, o, G); break; \
            case 2: hipLaunchKernelGGL((kern<F32, 2>), grid, dim3(256), 0, s, in, img, o, G); break; \
            default: hipLaunchKernelGGL((kern<F32, 1>), grid, dim3(256), 0, s, in, img, o, G); break; \
        }                                                                                  \
    }
MDP_SPEC_LAUNCH(spec_inv_kernel)
#undef MDP_SPEC_LAUNCH

template <bool F32>
static void launch_spec_fwd_kernel(const float* in, const typename Frag<F32>::T* img, float* o,
                                   int G, hipStream_t s, const LiftArgs& lift) {
    const int ch = spec_fields_per_wg(G);
    const dim3 grid((unsigned)((G + ch - 1) / ch));
    switch (ch) {
        case 8: hipLaunchKernelGGL((spec_fwd_kernel<F32, 8>), grid, dim3(256), 0, s, in, img, o, G, lift); break;
        case 4: hipLaunchKernelGGL((spec_fwd_kernel<F32, 4>), grid, dim3(256), 0, s, in, img, o, G, lift); break;
        case 2: hipLaunchKernelGGL((spec_fwd_kernel<F32, 2>), grid, dim3(256), 0, s, in, img, o, G, lift); break;
        default: hipLaunchKernelGGL((spec_fwd_kernel<F32, 1>), grid, dim3(256), 0, s, in, img, o, G, lift); break;
    }
}

void launch_spec_fwd(const float* v, const void* img, float* X, int G, int f32, hipStream_t s,
                     const LiftArgs& lift) {
    const float* f = reinterpret_cast<const float*>(img);
    if (f32)
        launch_spec_fwd_kernel<true>(v, f, X, G, s, lift);
    else
        launch_spec_fwd_kernel<false>(v, reinterpret_cast<const unsigned short*>(f + kImgElems),
                                      X, G, s, lift);
}
void launch_spec_inv(const float* Y, const void* img, float* U, int G, int f32, hipStream_t s) {
    const float* f = reinterpret_cast<const float*>(img);
    if (f32)
        launch_spec_inv_kernel<true>(Y, f, U, G, s);
    else
        launch_spec_inv_kernel<false>(Y, reinterpret_cast<const unsigned short*>(f + kImgElems),
                                      U, G, s);
}
void launch_proj_fused(const float* v, const float* P1, const float* c1, const float* P2,
                       const float* c2, float* out, float* h_out, int B, int P, int f32,
                       hipStream_t s) {
    dim3 grid((P + 63) / 64, B);
    if (f32)
        hipLaunchKernelGGL(proj_fused_kernel<true>, grid, dim3(256), 0, s, v, P1, c1, P2, c2,
                           out, h_out, P);
    else
        hipLaunchKernelGGL(proj_fused_kernel<false>, grid, dim3(256), 0, s, v, P1, c1, P2, c2,
                           out, h_out, P);
}
// the last pointwise layer fused with the projection head (32 channels,
// 128 hidden units, P a multiple of 64)
void launch_pointwise_proj(const float* W, const float* v, const float* bias, float* z,
                           int store_z, const float* P1, const float* c1, const float* P2,
                           const float* c2, float* out, float* h_out, int B, int P, int f32,
                           hipStream_t s) {
    dim3 grid(P / 64, B);
    if (f32)
        hipLaunchKernelGGL(pointwise_proj_kernel<true>, grid, dim3(256), 0, s, W, v, bias, z,
                           store_z, P1, c1, P2, c2, out, h_out, P);
    else
        hipLaunchKernelGGL(pointwise_proj_kernel<false>, grid, dim3(256), 0, s, W, v, bias, z,
                           store_z, P1, c1, P2, c2, out, h_out, P);
}
void launch_proj_back(const float* h, const float* P2, const float* gout, float* gh, int B,
                      int P, int K, hipStream_t s) {
    hipLaunchKernelGGL(proj_back_kernel, dim3(blocks_for((long long)B * K * P)), dim3(256), 0,
                       s, h, P2, gout, gh, B, P, K);
}
void launch_row_reduce(const float* x, const float* w, float* out, int B, int R, int P,
                       int mode, int accumulate, float* scratch, hipStream_t s) {
    if (scratch == nullptr || P % kRedCells != 0) {
        hipLaunchKernelGGL(row_reduce_kernel, dim3(R), dim3(256), 0, s, x, w, out, B, R, P,
                           mode, accumulate);
        return;
    }
    const int nch = B * (P / kRedCells);
    hipLaunchKernelGGL(row_reduce_part_kernel, dim3(R, nch), dim3(256), 0, s, x, w, scratch, R,
                       P, mode);
    hipLaunchKernelGGL(row_reduce_fin_kernel, dim3((R + 127) / 128), dim3(128), 0, s, scratch,
                       out, R, nch, accumulate);
}
void launch_lift_back(const float* in, const float* gv, float* gW0, float* gb0, int B, int n,
                      int C, float* scratch, hipStream_t s) {
    if (scratch == nullptr || (n * n) % kRedCells != 0) {
        hipLaunchKernelGGL(lift_back_kernel, dim3(C), dim3(256), 0, s, in, gv, gW0, gb0, B, n,
                           C);
        return;
    }
    const int nch = B * (n * n / kRedCells);
    hipLaunchKernelGGL(lift_back_part_kernel, dim3(C, nch), dim3(256), 0, s, in, gv, scratch, n,
                       C);
    hipLaunchKernelGGL(lift_back_fin_kernel, dim3((4 * C + 127) / 128), dim3(128), 0, s,
                       scratch, gW0, gb0, C, nch);
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
                          double* norms, int* active, RecastState* st, double tol, int k,
                          int B, int P, hipStream_t s) {
    hipLaunchKernelGGL(recast_update_kernel, dim3(B), dim3(256), 0, s, out, scale, inv_sa_star,
                       phi, norms, active, st, tol, k, P);
}
void launch_recast_average(const ResampleDesc* d, int B, int nc, float* S, float* sa,
                           hipStream_t s) {
    hipLaunchKernelGGL(recast_average_kernel, dim3((nc * nc + 255) / 256, B), dim3(256), 0, s,
                       d, nc, S, sa);
}
void launch_recast_output(const ResampleDesc* d, int B, int nc, long long max_cells,
                          const float* phi, hipStream_t s) {
    const long long g0 = (max_cells + 255) / 256, g = g0 < 4096 ? g0 : 4096;
    hipLaunchKernelGGL(recast_output_kernel, dim3((unsigned)g, B), dim3(256), 0, s, d, nc, phi);
}

}  // namespace mdp
