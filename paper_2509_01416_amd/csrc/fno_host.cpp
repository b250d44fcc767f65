// fno_host.cpp -- the network half of the C ABI: the 2-D Fourier neural
// operator of section 4.2 / Appendix A1 and the deep operator network of
// section 4.1 (model state, forward, hand-written backward, MSE + Adam
// training step) and the equation-recast loop of Eq. 24 that turns a
// trained network into an initial guess for source iteration.
//
// Every dense contraction goes through one batched matrix-core GEMM with
// strided views (launch_gemm).  The truncated 2-D real DFT of a 64 x 64
// channel is four small products with fixed matrices held on the device:
//   T  (64 x 24)  = v (64 y x 64 x) . FxT (64 x 24)       rfft along x
//   X  (48 x 12)  = Fy (48 x 128) . [T_re; T_im]           DFT along y
//   Z  (128 x 12) = Gy (128 x 48) . Y                      inverse along y
//   u  (64 x 64)  = Z' (64 y x 24) . Gx (24 x 64)          inverse rfft (x)
// with the retained modes kx in [0,12), ky in [0,12) U [52,64) and the 1/n^2
// and Hermitian factor c_kx (1 for kx = 0, else 2) folded into Gx.  The
// backward pass applies the transposes of the same matrices (read through
// transposed views), which is the exact adjoint of the forward map.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/mdpnop.h"
#include "eigen_kernels.h"
#include "fno_kernels.h"
#include "host_internal.h"

namespace mdp {

constexpr int kProj = 128;          // projection width (Appendix A1)
constexpr int kMaxBatch = 65535;    // samples per call (the batch is a grid dimension)
constexpr int kGridLog2 = 6;        // supported network grid 64 x 64
constexpr int kGrid = 1 << kGridLog2;
constexpr int kP = kGrid * kGrid;   // cells per field
constexpr int kPLog2 = 2 * kGridLog2;

struct FnoWork {
    Arena act;         // activations of the current batch
    Arena rc;          // recast-loop fields on the network grid
    PinnedBuf host;    // norm read-back
};

}  // namespace mdp

using namespace mdp;

// DeepONet shape (section 4.1, Appendix A1 carried to x-y): the 64 x 64
// grid as sensors, hidden width and basis size of the paper's networks.
constexpr int kDonHidden = 200, kDonBasis = 100;

struct no_model {
    int device = 0;
    int kind = 0;              // 0 Fourier neural operator, 1 DeepONet
    int width = 0, modes = 0, layers = 0, grid = 0;
    // DeepONet: parameter offsets, trunk input (cell centres [P][2]) and the
    // trunk activations t1, g1, t2, g2 [P][h] and basis [P][k], valid while
    // trunk_ver == param_ver (the basis depends on the parameters only)
    long long oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    long long oV1 = 0, oq1 = 0, oV2 = 0, oq2 = 0, oV3 = 0, oq3 = 0;
    float *coords = nullptr, *t1 = nullptr, *g1 = nullptr, *t2 = nullptr, *g2 = nullptr,
          *basis = nullptr;
    long long param_ver = 0, trunk_ver = -1;
    long long n_params = 0;
    long long oW0 = 0, ob0 = 0, oP1 = 0, oc1 = 0, oP2 = 0, oc2 = 0;
    std::vector<long long> oR, oW, ob;
    float* params = nullptr;   // FP32 master copy
    float* grad = nullptr;
    float* am = nullptr;       // Adam first moment
    float* av = nullptr;       // Adam second moment
    float* FxT = nullptr;      // [64][24]
    float* Fy = nullptr;       // [48][128]
    float* Gy = nullptr;       // [128][48]
    float* Gx = nullptr;       // [24][64]
    void* spec_img = nullptr;  // LDS images of the DFT matrices (mode window 12)
    long long step = 0;
    int f32 = 0;               // FP32 operands on the matrix cores
};

namespace {

// ------------------------------------------------------------ workspace --
struct Ws {
    int B = 0;
    std::vector<float*> v, z, X;   // layer inputs, pre-activations, kept modes
    float *h = nullptr, *T = nullptr, *Y = nullptr, *gX = nullptr;
    float *gv = nullptr, *gv2 = nullptr, *gz = nullptr, *gh = nullptr;
    float *out = nullptr, *gout = nullptr, *partial = nullptr, *rpart = nullptr;
    double* mse = nullptr;
    // DeepONet: branch pre-activations and activations [B][h], coefficients
    // [B][k]; training: their gradients, the basis gradient [P][k], trunk
    // gradients [P][h] and column-sum partials
    float *z1 = nullptr, *a1 = nullptr, *z2 = nullptr, *a2 = nullptr, *coef = nullptr;
    float *gcoef = nullptr, *gb = nullptr, *gz1 = nullptr, *gz2 = nullptr;
    float *gbasis = nullptr, *gtt = nullptr, *gt1 = nullptr, *gt2 = nullptr, *cpart = nullptr;
};

constexpr int kMaxKsplit = 1024;
constexpr int kMsePartials = 256;

// split-K partial buffer of the DeepONet's long contractions: K = P split
// in slices of 256 (16), times the largest M x N (a 200 x 200 weight, or a
// branch layer of at most kDonSplitBatch samples)
constexpr int kDonSplitBatch = 256;
constexpr long long kDonPartial = (long long)(kP / 256) *
                                  std::max(kDonHidden * kDonHidden, kDonSplitBatch * kDonHidden);
static_assert((kDonHidden + 31) / 32 <= kP / 256,
              "the split hidden layers fit the partial buffer");

size_t carve_don(int B, bool train, char* base, Ws* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    const size_t bh = 4 * (size_t)B * kDonHidden, bk = 4 * (size_t)B * kDonBasis;
    w->B = B;
    w->z1 = (float*)take(bh);
    w->a1 = (float*)take(bh);
    w->z2 = (float*)take(bh);
    w->a2 = (float*)take(bh);
    w->coef = (float*)take(bk);
    w->partial = (float*)take(4 * (size_t)kDonPartial);
    if (train) {
        w->gcoef = (float*)take(bk);
        w->gb = (float*)take(bh);
        w->gz1 = (float*)take(bh);
        w->gz2 = (float*)take(bh);
        w->gbasis = (float*)take(4 * (size_t)kP * kDonBasis);
        w->gtt = (float*)take(4 * (size_t)kP * kDonHidden);
        w->gt1 = (float*)take(4 * (size_t)kP * kDonHidden);
        w->gt2 = (float*)take(4 * (size_t)kP * kDonHidden);
        w->cpart = (float*)take(4 * (size_t)((std::max(kP, B) + kColChunk - 1) / kColChunk) *
                                kDonHidden);
        w->out = (float*)take(4 * (size_t)B * kP);
        w->gout = (float*)take(4 * (size_t)B * kP);
        w->mse = (double*)take(8 * kMsePartials);
    }
    return off;
}

size_t carve(const no_model* m, int B, bool train, char* base, Ws* w) {
    if (m->kind == 1) return carve_don(B, train, base, w);
    const long long C = m->width, L = m->layers, mm = m->modes;
    const long long act = (long long)B * C * kP;
    const long long modes = (long long)B * C * 2 * 2 * mm * mm;
    const long long tbuf = (long long)B * C * kGrid * 2 * mm;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    w->B = B;
    w->v.assign(L, nullptr);
    w->z.assign(L, nullptr);
    w->X.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
        w->v[l] = (float*)take(4 * act);
        w->z[l] = (float*)take(4 * act);
        w->X[l] = (float*)take(4 * modes);
    }
    w->T = (float*)take(4 * tbuf);
    w->Y = (float*)take(4 * modes);
    w->h = nullptr;
    if (train) {
        w->h = (float*)take(4 * (size_t)B * kProj * kP);
        w->gX = (float*)take(4 * modes);
        w->gv = (float*)take(4 * act);
        w->gv2 = (float*)take(4 * act);
        w->gz = (float*)take(4 * act);
        w->gh = (float*)take(4 * (size_t)B * kProj * kP);
        w->out = (float*)take(4 * (size_t)B * kP);
        w->gout = (float*)take(4 * (size_t)B * kP);
        w->partial = (float*)take(4 * (size_t)kMaxKsplit * C * kProj);
        w->rpart = (float*)take(4 * (size_t)4 * kProj * B * (kP / 1024));
        w->mse = (double*)take(8 * kMsePartials);
    }
    return off;
}

bool workspace(Ctx* c, const no_model* m, int B, bool train, Ws* w) {
    if (!c->fno) {
        c->fno = new (std::nothrow) FnoWork();
        if (!c->fno) {
            c->fail("out of host memory");
            return false;
        }
    }
    const size_t bytes = carve(m, B, train, nullptr, w);
    if (!c->fno->act.reserve(c, bytes)) return false;
    carve(m, B, train, (char*)c->fno->act.base, w);
    return true;
}

// ---------------------------------------------------------------- views --
View mat(const float* p, long long rs, long long cs, long long bs = 0) {
    View v;
    v.p = const_cast<float*>(p);
    v.sr_lo = rs;
    v.sc_lo = cs;
    v.sb_lo = bs;
    return v;
}

// The (p, y) x kx view of a [y][p][kx] buffer (p = re/im): row r = p*64 + y.
View tsplit(const float* p, int mm, long long bs) {
    View v = mat(p, 2 * mm, 1, bs);
    v.r_ls = kGridLog2;
    v.sr_hi = mm;
    v.sr_lo = 2 * mm;
    return v;
}

// Reduction over (batch, cell) as the K index of a [b][row][cell] tensor:
// K index kk = b * P + p.
View kcols(const float* p, long long rows_per_b) {   // A: (row, kk)
    View v = mat(p, kP, 1);
    v.c_ls = kPLog2;
    v.sc_hi = rows_per_b * kP;
    v.sc_lo = 1;
    return v;
}
View krows(const float* p, long long rows_per_b) {   // B: (kk, col)
    View v = mat(p, 1, kP);
    v.r_ls = kPLog2;
    v.sr_hi = rows_per_b * kP;
    v.sr_lo = 1;
    return v;
}

struct Runner {
    Ctx* c;
    const no_model* m;
    bool ok = true;

    bool gemm(int M, int N, int K, int G, View A, View B, View C, int acc = 0,
              const float* bias_row = nullptr, float* partial = nullptr,
              float* gelu_out = nullptr, const float* bias_col = nullptr,
              float* relu_out = nullptr, int ksplit = 0) {
        GemmArgs a;
        a.bias_col = bias_col;
        a.relu_out = relu_out;
        a.M = M;
        a.N = N;
        a.K = K;
        a.G = G;
        a.A = A;
        a.B = B;
        a.C = C;
        a.accumulate = acc;
        a.bias_row = bias_row;
        a.gelu_out = gelu_out;
        a.f32 = m->f32;
        if (partial && G == 1) {
            a.ksplit = std::max(1, std::min(kMaxKsplit, ksplit > 0 ? ksplit : K / 256));
            a.partial = partial;
        }
        if (!launch_gemm(a, c->stream)) {
            c->fail("gemm batch view cannot be chunked");
            ok = false;
        }
        return ok;
    }

    // DeepONet (section 4.1, Eq. 11).  Trunk on the P cell centres (kept on
    // the model until the parameters change), branch on the B sampled
    // inputs, then out[b][p] = sum_k coef[b][k] basis[p][k].
    void don_trunk() {
        const float* P = m->params;
        const int h = kDonHidden, k = kDonBasis;
        gemm(kP, h, 2, 1, mat(m->coords, 2, 1), mat(P + m->oV1, h, 1), mat(m->t1, h, 1), 0,
             nullptr, nullptr, nullptr, P + m->oq1, m->g1);
        gemm(kP, h, h, 1, mat(m->g1, h, 1), mat(P + m->oV2, h, 1), mat(m->t2, h, 1), 0,
             nullptr, nullptr, nullptr, P + m->oq2, m->g2);
        gemm(kP, k, h, 1, mat(m->g2, h, 1), mat(P + m->oV3, k, 1), mat(m->basis, k, 1), 0,
             nullptr, nullptr, nullptr, P + m->oq3);
    }

    void don_forward(const float* in, float* out, Ws& w, bool train) {
        const float* P = m->params;
        const int h = kDonHidden, k = kDonBasis, B = w.B;
        if (train || const_cast<no_model*>(m)->trunk_ver != m->param_ver) {
            don_trunk();
            const_cast<no_model*>(m)->trunk_ver = m->param_ver;
        }
        float* split = B <= kDonSplitBatch ? w.partial : nullptr;
        gemm(B, h, kP, 1, mat(in, kP, 1), mat(P + m->oW1, h, 1), mat(w.z1, h, 1), 0, nullptr,
             split, nullptr, P + m->ob1, w.a1);
        // the two 200-deep layers: one 32-wide K stage per workgroup (a
        // handful of output tiles would otherwise walk seven stages each)
        const int ks = (h + 31) / 32;
        gemm(B, h, h, 1, mat(w.a1, h, 1), mat(P + m->oW2, h, 1), mat(w.z2, h, 1), 0, nullptr,
             split, nullptr, P + m->ob2, w.a2, ks);
        gemm(B, k, h, 1, mat(w.a2, h, 1), mat(P + m->oW3, k, 1), mat(w.coef, k, 1), 0, nullptr,
             split, nullptr, P + m->ob3, nullptr, ks);
        gemm(B, kP, k, 1, mat(w.coef, k, 1), mat(m->basis, 1, k), mat(out, kP, 1));
    }

    // Gradient of sum(gout * out) into m->grad (every entry written).
    void don_backward(const float* in, const float* gout, Ws& w) {
        const float* P = m->params;
        float* g = m->grad;
        const int h = kDonHidden, k = kDonBasis, B = w.B;
        float* split = B <= kDonSplitBatch ? w.partial : nullptr;
        gemm(B, k, kP, 1, mat(gout, kP, 1), mat(m->basis, k, 1), mat(w.gcoef, k, 1), 0, nullptr,
             split);
        gemm(kP, k, B, 1, mat(gout, 1, kP), mat(w.coef, k, 1), mat(w.gbasis, k, 1));
        // branch
        gemm(h, k, B, 1, mat(w.a2, 1, h), mat(w.gcoef, k, 1), mat(g + m->oW3, k, 1));
        launch_col_sum(w.gcoef, g + m->ob3, B, k, w.cpart, c->stream);
        gemm(B, h, k, 1, mat(w.gcoef, k, 1), mat(P + m->oW3, 1, k), mat(w.gb, h, 1));
        launch_relu_back(w.z2, w.gb, w.gz2, (long long)B * h, c->stream);
        gemm(h, h, B, 1, mat(w.a1, 1, h), mat(w.gz2, h, 1), mat(g + m->oW2, h, 1));
        launch_col_sum(w.gz2, g + m->ob2, B, h, w.cpart, c->stream);
        gemm(B, h, h, 1, mat(w.gz2, h, 1), mat(P + m->oW2, 1, h), mat(w.gb, h, 1));
        launch_relu_back(w.z1, w.gb, w.gz1, (long long)B * h, c->stream);
        gemm(kP, h, B, 1, mat(in, 1, kP), mat(w.gz1, h, 1), mat(g + m->oW1, h, 1));
        launch_col_sum(w.gz1, g + m->ob1, B, h, w.cpart, c->stream);
        // trunk
        gemm(h, k, kP, 1, mat(m->g2, 1, h), mat(w.gbasis, k, 1), mat(g + m->oV3, k, 1), 0,
             nullptr, w.partial);
        launch_col_sum(w.gbasis, g + m->oq3, kP, k, w.cpart, c->stream);
        gemm(kP, h, k, 1, mat(w.gbasis, k, 1), mat(P + m->oV3, 1, k), mat(w.gtt, h, 1));
        launch_relu_back(m->t2, w.gtt, w.gt2, (long long)kP * h, c->stream);
        gemm(h, h, kP, 1, mat(m->g1, 1, h), mat(w.gt2, h, 1), mat(g + m->oV2, h, 1), 0, nullptr,
             w.partial);
        launch_col_sum(w.gt2, g + m->oq2, kP, h, w.cpart, c->stream);
        gemm(kP, h, h, 1, mat(w.gt2, h, 1), mat(P + m->oV2, 1, h), mat(w.gtt, h, 1));
        launch_relu_back(m->t1, w.gtt, w.gt1, (long long)kP * h, c->stream);
        gemm(2, h, kP, 1, mat(m->coords, 1, 2), mat(w.gt1, h, 1), mat(g + m->oV1, h, 1), 0,
             nullptr, w.partial);
        launch_col_sum(w.gt1, g + m->oq1, kP, h, w.cpart, c->stream);
    }

    // Forward of `B` fields in[b] ([B][P]) -> out ([B][P]); activations kept
    // in w for a following backward.
    void forward(const float* in, float* out, Ws& w, bool keep_h = false) {
        if (m->kind == 1) {
            don_forward(in, out, w, keep_h);
            return;
        }
        const int C = m->width, L = m->layers, mm = m->modes, B = w.B;
        const float* P = m->params;
        const int G = B * C;
        const long long act = (long long)C * kP;
        const long long per = 4LL * mm * mm, tb = (long long)kGrid * 2 * mm;
        // without a backward pass the first layer forms the lift where it
        // reads it (no stored v[0]); a backward pass needs the stored one
        const bool late_lift = !keep_h && C == 32 && mm == 12 && L >= 2;
        const LiftArgs lift0 = late_lift ? LiftArgs{in, P + m->oW0, P + m->ob0} : LiftArgs{};
        if (!late_lift) launch_lift(in, P + m->oW0, P + m->ob0, w.v[0], B, kGrid, C, c->stream);
        for (int l = 0; l < L && ok; ++l) {
            const LiftArgs lift = l == 0 ? lift0 : LiftArgs{};
            if (mm == 12) {   // the supported mode window: fused DFT kernels
                launch_spec_fwd(w.v[l], m->spec_img, w.X[l], G, m->f32, c->stream, lift);
                launch_mix(w.X[l], P + m->oR[l], w.Y, B, C, mm, c->stream);
                launch_spec_inv(w.Y, m->spec_img, w.z[l], G, m->f32, c->stream);
            } else {
                gemm(kGrid, 2 * mm, kGrid, G, mat(w.v[l], kGrid, 1, kP),
                     mat(m->FxT, 2 * mm, 1), mat(w.T, 2 * mm, 1, tb));
                gemm(4 * mm, mm, 2 * kGrid, G, mat(m->Fy, 2 * kGrid, 1), tsplit(w.T, mm, tb),
                     mat(w.X[l], mm, 1, per));
                launch_mix(w.X[l], P + m->oR[l], w.Y, B, C, mm, c->stream);
                gemm(2 * kGrid, mm, 4 * mm, G, mat(m->Gy, 4 * mm, 1), mat(w.Y, mm, 1, per),
                     tsplit(w.T, mm, tb));
                gemm(kGrid, kGrid, 2 * mm, G, mat(w.T, 2 * mm, 1, tb), mat(m->Gx, kGrid, 1),
                     mat(w.z[l], kGrid, 1, kP));
            }
            // pointwise path, bias and (but after the last layer) GELU; the
            // pre-activations are kept for a backward pass and for the head
            if (C == 32 && l + 1 == L) {
                // the last layer and the projection head in one kernel
                static_assert(kProj == 128, "the fused head has 128 hidden units");
                launch_pointwise_proj(P + m->oW[l], w.v[l], P + m->ob[l], w.z[l],
                                      keep_h ? 1 : 0, P + m->oP1, P + m->oc1, P + m->oP2,
                                      P + m->oc2, out, keep_h ? w.h : nullptr, B, kP, m->f32,
                                      c->stream);
                return;
            }
            if (C == 32) {
                launch_pointwise(P + m->oW[l], w.v[l], P + m->ob[l], w.z[l],
                                 l + 1 < L ? w.v[l + 1] : nullptr, B, kP,
                                 keep_h || l + 1 == L ? 1 : 0, m->f32, c->stream, lift);
            } else {
                gemm(C, kP, C, B, mat(P + m->oW[l], 1, C), mat(w.v[l], kP, 1, act),
                     mat(w.z[l], kP, 1, act), 1, P + m->ob[l], nullptr,
                     l + 1 < L ? w.v[l + 1] : nullptr);
            }
        }
        const float* vL = w.z[L - 1];
        // projection head; h is kept only when a backward pass follows
        launch_proj_fused(vL, P + m->oP1, P + m->oc1, P + m->oP2, P + m->oc2, out,
                          keep_h ? w.h : nullptr, B, kP, m->f32, c->stream);
    }

    // Gradient of sum(gout * out) into m->grad (every entry written).
    void backward(const float* in, const float* gout, Ws& w) {
        if (m->kind == 1) {
            don_backward(in, gout, w);
            return;
        }
        const int C = m->width, L = m->layers, mm = m->modes, B = w.B;
        const float* P = m->params;
        float* g = m->grad;
        const int G = B * C;
        const long long act = (long long)C * kP;
        const long long per = 4LL * mm * mm, tb = (long long)kGrid * 2 * mm;
        const float* vL = w.z[L - 1];
        launch_row_reduce(w.h, gout, g + m->oP2, B, kProj, kP, 2, 0, w.rpart, c->stream);
        launch_row_reduce(gout, nullptr, g + m->oc2, B, 1, kP, 0, 0, w.rpart, c->stream);
        launch_proj_back(w.h, P + m->oP2, gout, w.gh, B, kP, kProj, c->stream);
        gemm(C, kProj, B * kP, 1, kcols(vL, C), krows(w.gh, kProj), mat(g + m->oP1, kProj, 1),
             0, nullptr, w.partial);
        launch_row_reduce(w.gh, nullptr, g + m->oc1, B, kProj, kP, 0, 0, w.rpart, c->stream);
        gemm(C, kP, kProj, B, mat(P + m->oP1, kProj, 1), mat(w.gh, kP, 1, (long long)kProj * kP),
             mat(w.gv, kP, 1, act));
        float* gv = w.gv;
        float* gv2 = w.gv2;
        for (int l = L - 1; l >= 0 && ok; --l) {
            float* gz = gv;
            if (l + 1 < L) {
                launch_gelu_back(w.z[l], gv, w.gz, (long long)B * act, c->stream);
                gz = w.gz;
            }
            gemm(C, C, B * kP, 1, kcols(w.v[l], C), krows(gz, C), mat(g + m->oW[l], C, 1), 0,
                 nullptr, w.partial);
            launch_row_reduce(gz, nullptr, g + m->ob[l], B, C, kP, 0, 0, w.rpart, c->stream);
            gemm(C, kP, C, B, mat(P + m->oW[l], C, 1), mat(gz, kP, 1, act), mat(gv2, kP, 1, act));
            // spectral path, adjoint of the forward products
            gemm(kGrid, 2 * mm, kGrid, G, mat(gz, kGrid, 1, kP), mat(m->Gx, 1, kGrid),
                 mat(w.T, 2 * mm, 1, tb));
            gemm(4 * mm, mm, 2 * kGrid, G, mat(m->Gy, 1, 4 * mm), tsplit(w.T, mm, tb),
                 mat(w.Y, mm, 1, per));
            launch_mix_back_w(w.X[l], w.Y, g + m->oR[l], B, C, mm, c->stream);
            launch_mix_back_x(w.Y, P + m->oR[l], w.gX, B, C, mm, c->stream);
            gemm(2 * kGrid, mm, 4 * mm, G, mat(m->Fy, 1, 2 * kGrid), mat(w.gX, mm, 1, per),
                 tsplit(w.T, mm, tb));
            gemm(kGrid, kGrid, 2 * mm, G, mat(w.T, 2 * mm, 1, tb), mat(m->FxT, 1, 2 * mm),
                 mat(gv2, kGrid, 1, kP), 1);
            std::swap(gv, gv2);
        }
        launch_lift_back(in, gv, g + m->oW0, g + m->ob0, B, kGrid, C, w.rpart, c->stream);
    }
};

// DFT matrices of the retained modes (FP64 on the host, stored FP32).
void dft_matrices(int mm, std::vector<float>& FxT, std::vector<float>& Fy,
                  std::vector<float>& Gy, std::vector<float>& Gx) {
    const int n = kGrid, w2 = 2 * mm, ny = 2 * mm;
    const double tp = 2.0 * M_PI / n;
    FxT.assign((size_t)n * w2, 0.f);
    for (int x = 0; x < n; ++x)
        for (int k = 0; k < mm; ++k) {
            const long long ph = ((long long)k * x) % n;
            FxT[x * w2 + k] = (float)std::cos(tp * ph);
            FxT[x * w2 + mm + k] = (float)-std::sin(tp * ph);
        }
    Fy.assign((size_t)2 * ny * 2 * n, 0.f);
    Gy.assign((size_t)2 * n * 2 * ny, 0.f);
    for (int kyi = 0; kyi < ny; ++kyi) {
        const int ky = kyi < mm ? kyi : n - 2 * mm + kyi;
        for (int y = 0; y < n; ++y) {
            const long long ph = ((long long)ky * y) % n;
            const float cs = (float)std::cos(tp * ph), sn = (float)std::sin(tp * ph);
            // X = Fy [T_re; T_im]:  X_re = c T_re + s T_im, X_im = -s T_re + c T_im
            Fy[(size_t)(0 * ny + kyi) * 2 * n + 0 * n + y] = cs;
            Fy[(size_t)(0 * ny + kyi) * 2 * n + 1 * n + y] = sn;
            Fy[(size_t)(1 * ny + kyi) * 2 * n + 0 * n + y] = -sn;
            Fy[(size_t)(1 * ny + kyi) * 2 * n + 1 * n + y] = cs;
            // Z = Gy Y:  Z_re = c Y_re - s Y_im, Z_im = s Y_re + c Y_im
            Gy[(size_t)(0 * n + y) * 2 * ny + 0 * ny + kyi] = cs;
            Gy[(size_t)(0 * n + y) * 2 * ny + 1 * ny + kyi] = -sn;
            Gy[(size_t)(1 * n + y) * 2 * ny + 0 * ny + kyi] = sn;
            Gy[(size_t)(1 * n + y) * 2 * ny + 1 * ny + kyi] = cs;
        }
    }
    Gx.assign((size_t)w2 * n, 0.f);
    const double inv = 1.0 / ((double)n * n);
    for (int k = 0; k < mm; ++k) {
        const double ck = (k == 0 ? 1.0 : 2.0) * inv;
        for (int x = 0; x < n; ++x) {
            const long long ph = ((long long)k * x) % n;
            Gx[(size_t)k * n + x] = (float)(ck * std::cos(tp * ph));
            Gx[(size_t)(mm + k) * n + x] = (float)(-ck * std::sin(tp * ph));
        }
    }
}

void free_model(no_model* m) {
    float* bufs[] = {m->params, m->grad, m->am, m->av, m->FxT, m->Fy, m->Gy, m->Gx,
                     m->coords, m->t1, m->g1, m->t2, m->g2, m->basis};
    for (float* b : bufs)
        if (b) (void)hipFree(b);
    if (m->spec_img) (void)hipFree(m->spec_img);
}

bool same_device(Ctx* c, const no_model* m) {
    if (m->device != c->device) {
        c->fail("model lives on device %d, context on device %d", m->device, c->device);
        return false;
    }
    return true;
}

tr_status finish(Ctx* c, const char* what) {
    if (!c->hip_ok(hipGetLastError(), what)) return TR_ERR_HIP;
    if (!c->hip_ok(hipStreamSynchronize(c->stream), "sync")) return TR_ERR_HIP;
    return TR_OK;
}

tr_status ws_status(Ctx* c) {
    return c->err.rfind("out of", 0) == 0 ? TR_ERR_OOM : TR_ERR_INVALID_ARG;
}

}  // namespace

void mdp::Ctx::release_fno() {
    if (!fno) return;
    if (fno->act.base) (void)hipFree(fno->act.base);
    if (fno->rc.base) (void)hipFree(fno->rc.base);
    if (fno->host.ptr) (void)hipHostFree(fno->host.ptr);
    delete fno;
    fno = nullptr;
}

// ===================================================================== ABI

extern "C" tr_status no_model_create(tr_context* ctx, no_model** out, int32_t width,
                                     int32_t modes, int32_t layers, int32_t grid,
                                     const float* params_host) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c || !out) return TR_ERR_INVALID_ARG;
    c->err.clear();
    *out = nullptr;
    if (width != 32 || modes != 12 || layers != 4 || grid != kGrid) {
        c->fail("unsupported network shape (width %d, modes %d, layers %d, grid %d); "
                "supported: 32, 12, 4, 64", width, modes, layers, grid);
        return TR_ERR_INVALID_ARG;
    }
    no_model* m = new (std::nothrow) no_model();
    if (!m) return TR_ERR_OOM;
    m->device = c->device;
    m->width = width;
    m->modes = modes;
    m->layers = layers;
    m->grid = grid;
    long long o = 0;
    const long long w = width, mm = modes;
    m->oW0 = o; o += 3 * w;
    m->ob0 = o; o += w;
    for (int l = 0; l < layers; ++l) {
        m->oR.push_back(o); o += 2 * mm * mm * w * w * 2;
        m->oW.push_back(o); o += w * w;
        m->ob.push_back(o); o += w;
    }
    m->oP1 = o; o += w * kProj;
    m->oc1 = o; o += kProj;
    m->oP2 = o; o += kProj;
    m->oc2 = o; o += 1;
    m->n_params = o;
    std::vector<float> FxT, Fy, Gy, Gx;
    dft_matrices(modes, FxT, Fy, Gy, Gx);
    const size_t pb = sizeof(float) * (size_t)o;
    bool good = c->hip_ok(hipMalloc(&m->params, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->grad, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->am, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->av, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->FxT, 4 * FxT.size()), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->Fy, 4 * Fy.size()), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->Gy, 4 * Gy.size()), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->Gx, 4 * Gx.size()), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->spec_img, spec_image_bytes()), "hipMalloc");
    if (good) {
        hipStream_t s = c->stream;
        good = (params_host
                    ? c->hip_ok(hipMemcpyAsync(m->params, params_host, pb, hipMemcpyHostToDevice, s),
                                "copy")
                    : c->hip_ok(hipMemsetAsync(m->params, 0, pb, s), "memset")) &&
               c->hip_ok(hipMemsetAsync(m->grad, 0, pb, s), "memset") &&
               c->hip_ok(hipMemsetAsync(m->am, 0, pb, s), "memset") &&
               c->hip_ok(hipMemsetAsync(m->av, 0, pb, s), "memset") &&
               c->hip_ok(hipMemcpyAsync(m->FxT, FxT.data(), 4 * FxT.size(), hipMemcpyHostToDevice, s), "copy") &&
               c->hip_ok(hipMemcpyAsync(m->Fy, Fy.data(), 4 * Fy.size(), hipMemcpyHostToDevice, s), "copy") &&
               c->hip_ok(hipMemcpyAsync(m->Gy, Gy.data(), 4 * Gy.size(), hipMemcpyHostToDevice, s), "copy") &&
               c->hip_ok(hipMemcpyAsync(m->Gx, Gx.data(), 4 * Gx.size(), hipMemcpyHostToDevice, s), "copy");
        if (good && modes == 12 && grid == kGrid) {
            launch_stage_spec(m->FxT, m->Fy, m->Gy, m->Gx, m->spec_img, s);
            good = c->hip_ok(hipGetLastError(), "stage launch");
        }
        good = good && c->hip_ok(hipStreamSynchronize(s), "sync");
    }
    if (!good) {
        (void)hipGetLastError();
        free_model(m);
        delete m;
        return c->err.find("out of memory") != std::string::npos ? TR_ERR_OOM : TR_ERR_HIP;
    }
    *out = m;
    return TR_OK;
}

extern "C" tr_status no_model_create_deeponet(tr_context* ctx, no_model** out, int32_t grid,
                                              int32_t hidden, int32_t basis,
                                              const float* params_host) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c || !out) return TR_ERR_INVALID_ARG;
    c->err.clear();
    *out = nullptr;
    if (grid != kGrid || hidden != kDonHidden || basis != kDonBasis) {
        c->fail("unsupported DeepONet shape (grid %d, hidden %d, basis %d); supported: "
                "%d, %d, %d", grid, hidden, basis, kGrid, kDonHidden, kDonBasis);
        return TR_ERR_INVALID_ARG;
    }
    no_model* m = new (std::nothrow) no_model();
    if (!m) return TR_ERR_OOM;
    m->device = c->device;
    m->kind = 1;
    m->grid = grid;
    const long long s_ = kP, d = 2, h = hidden, k = basis;
    long long o = 0;
    m->oW1 = o; o += s_ * h;
    m->ob1 = o; o += h;
    m->oW2 = o; o += h * h;
    m->ob2 = o; o += h;
    m->oW3 = o; o += h * k;
    m->ob3 = o; o += k;
    m->oV1 = o; o += d * h;
    m->oq1 = o; o += h;
    m->oV2 = o; o += h * h;
    m->oq2 = o; o += h;
    m->oV3 = o; o += h * k;
    m->oq3 = o; o += k;
    m->n_params = o;
    const size_t pb = sizeof(float) * (size_t)o;
    const size_t th = sizeof(float) * (size_t)kP * h;
    bool good = c->hip_ok(hipMalloc(&m->params, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->grad, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->am, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->av, pb), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->coords, sizeof(float) * 2 * kP), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->t1, th), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->g1, th), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->t2, th), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->g2, th), "hipMalloc") &&
                c->hip_ok(hipMalloc(&m->basis, sizeof(float) * (size_t)kP * k), "hipMalloc");
    if (good) {
        hipStream_t s = c->stream;
        good = (params_host
                    ? c->hip_ok(hipMemcpyAsync(m->params, params_host, pb, hipMemcpyHostToDevice, s),
                                "copy")
                    : c->hip_ok(hipMemsetAsync(m->params, 0, pb, s), "memset")) &&
               c->hip_ok(hipMemsetAsync(m->grad, 0, pb, s), "memset") &&
               c->hip_ok(hipMemsetAsync(m->am, 0, pb, s), "memset") &&
               c->hip_ok(hipMemsetAsync(m->av, 0, pb, s), "memset");
        if (good) {
            launch_grid_coords(m->coords, kGrid, s);
            good = c->hip_ok(hipGetLastError(), "coords launch");
        }
        good = good && c->hip_ok(hipStreamSynchronize(s), "sync");
    }
    if (!good) {
        (void)hipGetLastError();
        free_model(m);
        delete m;
        return TR_ERR_HIP;
    }
    *out = m;
    return TR_OK;
}

extern "C" void no_model_destroy(no_model* m) {
    if (!m) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != m->device) (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    free_model(m);
    if (cur != m->device) (void)hipSetDevice(cur);
    delete m;
}

extern "C" int64_t no_model_param_count(const no_model* m) { return m ? m->n_params : 0; }

extern "C" tr_status no_model_set_fp32(no_model* m, int32_t enable) {
    if (!m || (enable != 0 && enable != 1)) return TR_ERR_INVALID_ARG;
    m->f32 = enable;
    return TR_OK;
}

extern "C" tr_status no_model_get_params(tr_context* ctx, const no_model* m, float* params_host) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!m || !params_host) {
        c->fail("null model or buffer");
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    if (!c->hip_ok(hipMemcpyAsync(params_host, m->params, 4 * (size_t)m->n_params,
                                  hipMemcpyDeviceToHost, c->stream), "copy"))
        return TR_ERR_HIP;
    return finish(c, "get params");
}

extern "C" tr_status no_model_set_params(tr_context* ctx, no_model* m, const float* params_host) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!m || !params_host) {
        c->fail("null model or buffer");
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    const size_t pb = 4 * (size_t)m->n_params;
    if (!c->hip_ok(hipMemcpyAsync(m->params, params_host, pb, hipMemcpyHostToDevice, c->stream),
                   "copy") ||
        !c->hip_ok(hipMemsetAsync(m->am, 0, pb, c->stream), "memset") ||
        !c->hip_ok(hipMemsetAsync(m->av, 0, pb, c->stream), "memset"))
        return TR_ERR_HIP;
    m->step = 0;
    m->param_ver += 1;
    return finish(c, "set params");
}

extern "C" tr_status no_model_get_state(tr_context* ctx, const no_model* m, float* params_host,
                                        float* adam_m_host, float* adam_v_host,
                                        int64_t* step) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!m || !params_host || !adam_m_host || !adam_v_host || !step) {
        c->fail("null model, buffer or step");
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    const size_t pb = 4 * (size_t)m->n_params;
    if (!c->hip_ok(hipMemcpyAsync(params_host, m->params, pb, hipMemcpyDeviceToHost, c->stream),
                   "copy") ||
        !c->hip_ok(hipMemcpyAsync(adam_m_host, m->am, pb, hipMemcpyDeviceToHost, c->stream),
                   "copy") ||
        !c->hip_ok(hipMemcpyAsync(adam_v_host, m->av, pb, hipMemcpyDeviceToHost, c->stream),
                   "copy"))
        return TR_ERR_HIP;
    const tr_status st = finish(c, "get state");
    if (st == TR_OK) *step = m->step;
    return st;
}

extern "C" tr_status no_model_set_state(tr_context* ctx, no_model* m, const float* params_host,
                                        const float* adam_m_host, const float* adam_v_host,
                                        int64_t step) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!m || !params_host || !adam_m_host || !adam_v_host || step < 0) {
        c->fail("null model or buffer, or a negative step count");
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    const size_t pb = 4 * (size_t)m->n_params;
    if (!c->hip_ok(hipMemcpyAsync(m->params, params_host, pb, hipMemcpyHostToDevice, c->stream),
                   "copy") ||
        !c->hip_ok(hipMemcpyAsync(m->am, adam_m_host, pb, hipMemcpyHostToDevice, c->stream),
                   "copy") ||
        !c->hip_ok(hipMemcpyAsync(m->av, adam_v_host, pb, hipMemcpyHostToDevice, c->stream),
                   "copy"))
        return TR_ERR_HIP;
    m->param_ver += 1;
    const tr_status st = finish(c, "set state");
    if (st == TR_OK) m->step = step;
    return st;
}

extern "C" tr_status no_forward(tr_context* ctx, const no_model* m, int32_t batch,
                                const float* input, float* output) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!m || batch <= 0 || batch > kMaxBatch || !input || !output) {
        c->fail("no_forward: need a model, 0 < batch <= %d and buffers", kMaxBatch);
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    Ws w;
    if (!workspace(c, m, batch, false, &w)) return ws_status(c);
    Runner r{c, m};
    r.forward(input, output, w);
    if (!r.ok) return TR_ERR_INVALID_ARG;
    return finish(c, "forward launch");
}

extern "C" tr_status no_train_step(tr_context* ctx, no_model* m, int32_t batch,
                                   const float* input, const float* target, double lr,
                                   double* loss, float* grad_out) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    if (!m || batch <= 0 || batch > kMaxBatch || !input || !target || !(lr >= 0.0) ||
        !std::isfinite(lr)) {
        c->fail("no_train_step: need a model, 0 < batch <= %d, buffers and a finite lr >= 0",
                kMaxBatch);
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    Ws w;
    if (!workspace(c, m, batch, true, &w)) return ws_status(c);
    if (!c->fno->host.reserve(c, sizeof(double) * kMsePartials)) return ws_status(c);
    Runner r{c, m};
    r.forward(input, w.out, w, true);
    const long long n = (long long)batch * kP;
    const int nb = launch_mse(w.out, target, w.gout, w.mse, n, c->stream);
    r.backward(input, w.gout, w);
    if (!r.ok) return TR_ERR_INVALID_ARG;
    if (grad_out &&
        !c->hip_ok(hipMemcpyAsync(grad_out, m->grad, 4 * (size_t)m->n_params,
                                  hipMemcpyDeviceToDevice, c->stream), "copy"))
        return TR_ERR_HIP;
    if (lr > 0.0) {
        m->step += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 - std::pow(b1, (double)m->step));
        const float c2 = (float)(1.0 - std::pow(b2, (double)m->step));
        launch_adam(m->params, m->grad, m->am, m->av, m->n_params, (float)lr, (float)b1,
                    (float)b2, 1e-8f, c1, c2, c->stream);
        m->param_ver += 1;
    }
    double* hp = (double*)c->fno->host.ptr;
    if (!c->hip_ok(hipMemcpyAsync(hp, w.mse, sizeof(double) * nb, hipMemcpyDeviceToHost,
                                  c->stream), "copy"))
        return TR_ERR_HIP;
    const tr_status st = finish(c, "train launch");
    if (st != TR_OK) return st;
    double s = 0.0;
    for (int i = 0; i < nb; ++i) s += hp[i];
    if (loss) *loss = s / (double)n;
    if (!std::isfinite(s)) {
        c->fail("non-finite loss");
        return TR_ERR_NONFINITE;
    }
    return TR_OK;
}

extern "C" tr_status no_recast_guess(tr_context* ctx, const no_model* m, int32_t n_inst,
                                     const tr_problem* p, double sigma_t_star,
                                     double sigma_s_star, double tol, int32_t max_iter,
                                     float* const* phi_guess, tr_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!m || !phi_guess) {
        c->fail("no_recast_guess: need a model and output pointers");
        return TR_ERR_INVALID_ARG;
    }
    if (n_inst > kMaxBatch) {
        c->fail("no_recast_guess: at most %d problems per call", kMaxBatch);
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    if (!check_problems(c, n_inst, p, true)) return TR_ERR_INVALID_ARG;
    const double sa_star = sigma_t_star - sigma_s_star;
    if (!(sa_star > 0.0) || !std::isfinite(sa_star) || !(sigma_s_star >= 0.0)) {
        c->fail("need sigma_t* > sigma_s* >= 0 (finite)");
        return TR_ERR_INVALID_ARG;
    }
    if (!(tol >= 0.0) || !std::isfinite(tol) || max_iter < 1) {
        c->fail("need tol >= 0 and max_iter >= 1");
        return TR_ERR_INVALID_ARG;
    }
    std::vector<int> fac(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        const tr_problem& P = p[i];
        if (P.dim != 2 || P.nx != P.ny || P.nx % kGrid != 0 || !phi_guess[i]) {
            c->fail("problem %d: need a 2-D square grid that is a multiple of %d and an "
                    "output pointer", i, kGrid);
            return TR_ERR_INVALID_ARG;
        }
        fac[i] = P.nx / kGrid;
    }
    const int B = n_inst;
    Ws w;
    if (!workspace(c, m, B, false, &w)) return ws_status(c);
    FnoWork* fw = c->fno;
    // recast fields: S, sigma_a, phi, in, out (B x P), scale (B), norms (2B),
    // active (B), loop state (B), resampling descriptors (B)
    const size_t fb = align_up(4 * (size_t)B * kP);
    const size_t dsz = align_up(sizeof(ResampleDesc) * (size_t)B);
    const size_t ssz = align_up(sizeof(RecastState) * (size_t)B);
    const size_t need = 5 * fb + align_up(4 * (size_t)B) + align_up(16 * (size_t)B) +
                        align_up(4 * (size_t)B) + ssz + dsz;
    const size_t hoff = align_up(16 * (size_t)B + 4 * (size_t)B);
    if (!fw->rc.reserve(c, need) || !fw->host.reserve(c, hoff + ssz + dsz))
        return ws_status(c);
    char* base = (char*)fw->rc.base;
    float* S = (float*)base;
    float* sa = (float*)(base + fb);
    float* phi = (float*)(base + 2 * fb);
    float* in = (float*)(base + 3 * fb);
    float* out = (float*)(base + 4 * fb);
    float* scale = (float*)(base + 5 * fb);
    double* norms = (double*)(base + 5 * fb + align_up(4 * (size_t)B));
    int* active = (int*)(base + 5 * fb + align_up(4 * (size_t)B) + align_up(16 * (size_t)B));
    RecastState* dst = (RecastState*)(base + 5 * fb + align_up(4 * (size_t)B) +
                                      align_up(16 * (size_t)B) + align_up(4 * (size_t)B));
    ResampleDesc* ddesc = (ResampleDesc*)((char*)dst + ssz);
    double* hn = (double*)fw->host.ptr;
    int* hact = (int*)(hn + 2 * B);
    RecastState* hst = (RecastState*)((char*)fw->host.ptr + hoff);
    ResampleDesc* hdesc = (ResampleDesc*)((char*)hst + ssz);
    hipStream_t s = c->stream;
    long long max_cells = 0;
    for (int i = 0; i < B; ++i) {
        hdesc[i] = ResampleDesc{p[i].sigma_t, p[i].sigma_s, p[i].source, phi_guess[i],
                                p[i].nx, fac[i]};
        max_cells = std::max(max_cells, (long long)p[i].nx * p[i].nx);
        hact[i] = 1;
        hst[i] = RecastState{0.0, 0.0, 0.0, {0.0, 0.0, 0.0, 0.0}, kRecastRunning, 0, 0, 0};
    }
    static_assert(kRecastConverged == TR_OK && kRecastRunning == TR_NOT_CONVERGED &&
                      kRecastDiverged == TR_RECAST_DIVERGED,
                  "recast status codes follow tr_status");
    if (!c->hip_ok(hipMemcpyAsync(ddesc, hdesc, sizeof(ResampleDesc) * (size_t)B,
                                  hipMemcpyHostToDevice, s), "copy") ||
        !c->hip_ok(hipMemcpyAsync(dst, hst, sizeof(RecastState) * (size_t)B,
                                  hipMemcpyHostToDevice, s), "copy"))
        return TR_ERR_HIP;
    launch_recast_average(ddesc, B, kGrid, S, sa, s);
    if (!c->hip_ok(hipMemsetAsync(phi, 0, 4 * (size_t)B * kP, s), "memset") ||
        !c->hip_ok(hipMemcpyAsync(active, hact, 4 * (size_t)B, hipMemcpyHostToDevice, s), "copy"))
        return TR_ERR_HIP;
    // The rules run on the device after every update (recast_update_kernel),
    // so several updates go out between read-backs of the loop state: two
    // first, then as many as the slowest running instance is predicted to
    // need from its last two relative changes (at most 8).  Updates enqueued
    // after every instance has stopped skip the per-instance kernels; only
    // their network forward is spent.
    int live = B, k = 0, chunk = 2;
    Runner r{c, m};
    while (k < max_iter && live > 0) {
        const int n = std::min(chunk, max_iter - k);
        for (int j = 0; j < n; ++j, ++k) {
            launch_recast_input(S, sa, phi, (float)sa_star, in, scale, active, B, kP, s);
            r.forward(in, out, w);
            if (!r.ok) return TR_ERR_INVALID_ARG;
            launch_recast_update(out, scale, (float)(1.0 / sa_star), phi, norms, active, dst,
                                 tol, k, B, kP, s);
        }
        // the guesses on the problems' grids as they stand: final when this
        // chunk ends the loop (saves a read-back), rewritten otherwise
        launch_recast_output(ddesc, B, kGrid, max_cells, phi, s);
        if (!c->hip_ok(hipMemcpyAsync(hst, dst, sizeof(RecastState) * (size_t)B,
                                      hipMemcpyDeviceToHost, s), "copy") ||
            !c->hip_ok(hipMemcpyAsync(hact, active, 4 * (size_t)B, hipMemcpyDeviceToHost, s),
                       "copy"))
            return TR_ERR_HIP;
        const tr_status st = finish(c, "recast launch");
        if (st != TR_OK) return st;
        live = 0;
        int want = 1;
        for (int b = 0; b < B; ++b) {
            if (!hact[b]) continue;
            ++live;
            const double d = hst[b].resid;
            const double d0 = k >= 2 ? hst[b].dh[(k - 2) & 3] : 0.0;
            int nb = 1;
            if (d > 0.0 && d0 > d && tol > 0.0) {
                const double left = std::log(tol / d) / std::log(d / d0);
                nb = left >= 8.0 ? 8 : std::max(1, (int)std::ceil(left));
            }
            want = std::max(want, nb);
        }
        chunk = want;
    }
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = TR_OK;
    for (int i = 0; i < B; ++i) {
        worst = std::max(worst, hst[i].status);
        if (stats) {
            stats[i].status = hst[i].status;
            stats[i].iterations = hst[i].iters;
            stats[i].residual = hst[i].resid;
            stats[i].balance_rel = NAN;
            stats[i].seconds = secs;
        }
    }
    return (tr_status)worst;
}

// ----------------------------------------------------------- no_eigen ----
// The neural-operator outer loop of the k-eigenvalue problem (Appendix A2,
// simple preconditioning Eq. A5 and constrained preconditioning Eq. A7-A8)
// on the network's own grid.  Per outer update and instance:
//   u = NO[ S + (sigma_a* - sigma_a) phi ],  S = nu_sigma_f phi / k   (Eq. A5 / A7)
//   CP only: u <- Sweep(sigma_s u + nu_sigma_f u / k)                    (Eq. A8)
// then the outer update P of eigen.hip (k, normalisation, convergence).
namespace mdp {
void launch_combine(int nblocks, const InstDesc* insts, const int4* blocks, const int* done,
                    double2* red, int mode, int norm_kind, hipStream_t s, const DirTable* dt);
}

extern "C" tr_status no_eigen(tr_context* ctx, const no_model* m, int32_t n_inst,
                              const tr_problem* p, const float* const* nu_sigma_f,
                              const tr_quadrature* q, double sigma_t_star, double sigma_s_star,
                              int32_t variant, const float* const* phi_init,
                              float* const* phi_out, const double* k_init, double tol_k,
                              double tol_phi, int32_t max_outer, tr_eigen_stats* stats) {
    Ctx* c = reinterpret_cast<Ctx*>(ctx);
    if (!c) return TR_ERR_INVALID_ARG;
    c->err.clear();
    const auto t0 = std::chrono::steady_clock::now();
    if (!m || !p || !nu_sigma_f || !phi_out || n_inst <= 0) {
        c->fail("no_eigen: need a model, n_inst > 0 problems, nu_sigma_f and phi_out");
        return TR_ERR_INVALID_ARG;
    }
    if (n_inst > kMaxBatch) {
        c->fail("no_eigen: at most %d problems per call", kMaxBatch);
        return TR_ERR_INVALID_ARG;
    }
    if (variant != NO_EIGEN_SP && variant != NO_EIGEN_CP) {
        c->fail("no_eigen: variant must be NO_EIGEN_SP or NO_EIGEN_CP");
        return TR_ERR_INVALID_ARG;
    }
    if (!(tol_k > 0.0) || !(tol_phi > 0.0) || !std::isfinite(tol_k) ||
        !std::isfinite(tol_phi) || max_outer <= 0) {
        c->fail("no_eigen: need finite tol_k, tol_phi > 0 and max_outer > 0");
        return TR_ERR_INVALID_ARG;
    }
    if (!same_device(c, m)) return TR_ERR_INVALID_ARG;
    const double sa_star = sigma_t_star - sigma_s_star;
    if (!(sa_star > 0.0) || !std::isfinite(sa_star) || !(sigma_s_star >= 0.0)) {
        c->fail("need sigma_t* > sigma_s* >= 0 (finite)");
        return TR_ERR_INVALID_ARG;
    }
    const int B = n_inst;
    std::vector<tr_problem> pp(p, p + B);
    for (int i = 0; i < B; ++i) {
        const tr_problem& P = p[i];
        if (P.dim != 2 || P.nx != kGrid || P.ny != kGrid || !nu_sigma_f[i] || !phi_out[i]) {
            c->fail("problem %d: no_eigen needs a 2-D %d x %d grid (the network's), "
                    "nu_sigma_f and phi_out", i, kGrid, kGrid);
            return TR_ERR_INVALID_ARG;
        }
        for (int f = 0; f < 4; ++f)
            if (P.bc[f] != TR_BC_VACUUM) {
                c->fail("problem %d: no_eigen needs vacuum faces", i);
                return TR_ERR_INVALID_ARG;
            }
        if (k_init && (!(k_init[i] > 0.0) || !std::isfinite(k_init[i]))) {
            c->fail("problem %d: k_init must be positive and finite", i);
            return TR_ERR_INVALID_ARG;
        }
        pp[i].source = P.sigma_t;   // placeholder for the check
    }
    if (!check_problems(c, B, pp.data(), true) || reject_anisotropic(c, B, pp.data(), "no_eigen"))
        return TR_ERR_INVALID_ARG;
    Ws w;
    if (!workspace(c, m, B, false, &w)) return ws_status(c);
    FnoWork* fw = c->fno;
    // fields (B x P each): nu_sigma_f, sigma_a, phi, in, out, S, Q, prev;
    // then scale (B), norms (2B), active (B), resampling descriptors (B),
    // eigen descriptors (B), eigen state (B), done flags (B)
    const size_t fb = align_up(4 * (size_t)B * kP);
    size_t off = 8 * fb;
    const size_t oScale = off;
    off += align_up(4 * (size_t)B);
    const size_t oNorm = off;
    off += align_up(16 * (size_t)B);
    const size_t oAct = off;
    off += align_up(4 * (size_t)B);
    const size_t oRd = off;
    off += align_up(sizeof(ResampleDesc) * (size_t)B);
    const size_t oEd = off;
    off += align_up(sizeof(EigDesc) * (size_t)B);
    const size_t oEs = off;
    off += align_up(sizeof(EigState) * (size_t)B);
    const size_t oDone = off;
    off += align_up(4 * (size_t)B);
    const size_t hRd = 0, hAct = align_up(sizeof(ResampleDesc) * (size_t)B),
                 hDone = hAct + align_up(4 * (size_t)B), hEnd = hDone + align_up(4 * (size_t)B);
    if (!fw->rc.reserve(c, off) || !fw->host.reserve(c, hEnd)) return ws_status(c);
    char* base = (char*)fw->rc.base;
    float* nsfb = (float*)base;
    float* sa = (float*)(base + fb);
    float* phi = (float*)(base + 2 * fb);
    float* in = (float*)(base + 3 * fb);
    float* out = (float*)(base + 4 * fb);
    float* Sf = (float*)(base + 5 * fb);
    float* Q = (float*)(base + 6 * fb);
    float* prev = (float*)(base + 7 * fb);
    float* scale = (float*)(base + oScale);
    double* norms = (double*)(base + oNorm);
    int* active = (int*)(base + oAct);
    ResampleDesc* ddesc = (ResampleDesc*)(base + oRd);
    EigDesc* d_ed = (EigDesc*)(base + oEd);
    EigState* d_es = (EigState*)(base + oEs);
    int* d_done = (int*)(base + oDone);
    char* hb = (char*)fw->host.ptr;
    ResampleDesc* hdesc = (ResampleDesc*)(hb + hRd);
    int* hact = (int*)(hb + hAct);
    int* hdone = (int*)(hb + hDone);
    hipStream_t s = c->stream;
    if (!c->hip_ok(hipStreamSynchronize(s), "sync")) return TR_ERR_HIP;
    // nu_sigma_f and sigma_a gathered into the batch layout (f = 1: copies)
    for (int i = 0; i < B; ++i)
        hdesc[i] = ResampleDesc{p[i].sigma_t, p[i].sigma_s, nu_sigma_f[i], phi_out[i], kGrid, 1};
    if (!c->hip_ok(hipMemcpyAsync(ddesc, hdesc, sizeof(ResampleDesc) * (size_t)B,
                                  hipMemcpyHostToDevice, s), "copy"))
        return TR_ERR_HIP;
    launch_recast_average(ddesc, B, kGrid, nsfb, sa, s);
    // the sweep's view of the batch: iterate phi, emission Q, source S
    std::vector<float*> phis(B), Qs(B);
    for (int i = 0; i < B; ++i) {
        phis[i] = phi + (size_t)i * kP;
        Qs[i] = Q + (size_t)i * kP;
        pp[i].source = Sf + (size_t)i * kP;
    }
    Setup su;
    if (!c->setup(B, pp.data(), q, nullptr, phis.data(), Qs.data(), &su))
        return c->err.rfind("out of", 0) == 0 ? TR_ERR_OOM : TR_ERR_INVALID_ARG;
    const size_t htab = oDone + align_up(4 * (size_t)B) - oEd;
    if (!c->hip_ok(hipStreamSynchronize(s), "sync")) return TR_ERR_HIP;
    if (!c->pinned.reserve(c, htab)) return TR_ERR_OOM;
    char* h = (char*)c->pinned.ptr;
    std::memset(h, 0, htab);
    EigDesc* hd = (EigDesc*)h;
    EigState* hs = (EigState*)(h + (oEs - oEd));
    for (int i = 0; i < B; ++i) {
        hd[i].nsf = nsfb + (size_t)i * kP;
        hd[i].phi0 = phi_init ? phi_init[i] : nullptr;
        hd[i].S = Sf + (size_t)i * kP;
        hd[i].prev = prev + (size_t)i * kP;
        hd[i].vol = su.inst[i].dx * su.inst[i].dy;
        hs[i].k = k_init ? k_init[i] : 1.0;
        hs[i].status = 1;
    }
    if (!c->hip_ok(hipMemcpyAsync(d_ed, h, htab, hipMemcpyHostToDevice, s), "copy") ||
        !c->hip_ok(hipMemsetAsync(su.st.iter, 0, sizeof(int) * B, s), "memset") ||
        !c->hip_ok(hipMemsetAsync(su.st.status, 0, sizeof(int) * B, s), "memset"))
        return TR_ERR_HIP;
    const int nblocks = (int)su.blocks.size();
    launch_eig_start(B, 1, nblocks, su.d_inst, su.d_blocks, d_ed, d_es, d_done, su.d_bpart, s);
    if (!c->hip_ok(hipMemcpyAsync(h, d_es, sizeof(EigState) * B, hipMemcpyDeviceToHost, s),
                   "copy"))
        return TR_ERR_HIP;
    tr_status st0 = finish(c, "eigen start");
    if (st0 != TR_OK) return st0;
    for (int i = 0; i < B; ++i) {
        if (((EigState*)h)[i].status < 0) {
            c->fail("problem %d: nu_sigma_f must be finite and >= 0 and the starting "
                    "flux finite with F(phi) > 0", i);
            return TR_ERR_INVALID_ARG;
        }
        hact[i] = 1;
    }
    // the cross-section checks of tr_eigen (finite, sigma_t > 0,
    // 0 <= sigma_s <= sigma_t), now that the start has defined the source
    {
        const tr_status sf = c->scan_fields(su, B, pp.data(), true, nullptr);
        if (sf != TR_OK) return sf;
    }
    if (!c->hip_ok(hipMemcpyAsync(active, hact, 4 * (size_t)B, hipMemcpyHostToDevice, s), "copy"))
        return TR_ERR_HIP;
    Runner r{c, m};
    for (int outer = 1; outer <= max_outer; ++outer) {
        launch_recast_input(Sf, sa, phi, (float)sa_star, in, scale, active, B, kP, s);
        r.forward(in, out, w);
        if (!r.ok) return TR_ERR_INVALID_ARG;
        launch_recast_update(out, scale, (float)(1.0 / sa_star), phi, norms, active, nullptr,
                             0.0, 0, B, kP, s);
        if (variant == NO_EIGEN_CP) {
            launch_eig_emission(nblocks, su.d_inst, su.d_blocks, d_ed, d_es, d_done, s);
            if (!c->launch_sweep(su, B, d_done, nullptr, 0)) return TR_ERR_HIP;
            launch_combine(nblocks, su.d_inst, su.d_blocks, d_done, su.d_red, 1, 0, s, su.d_dt);
        }
        launch_eig_update(B, 1, nblocks, su.d_inst, su.d_blocks, d_ed, d_es, d_done, su.d_bpart,
                          su.st, tol_k, tol_phi, outer == max_outer ? 1 : 0, s);
        if (!c->hip_ok(hipMemcpyAsync(hdone, d_done, 4 * (size_t)B, hipMemcpyDeviceToHost, s),
                       "copy"))
            return TR_ERR_HIP;
        const tr_status st = finish(c, "no_eigen outer");
        if (st != TR_OK) return st;
        bool all = true, changed = false;
        for (int i = 0; i < B; ++i) {
            all &= hdone[i] != 0;
            if (hdone[i] && hact[i]) {
                hact[i] = 0;
                changed = true;
            }
        }
        if (all) break;
        if (changed && !c->hip_ok(hipMemcpyAsync(active, hact, 4 * (size_t)B,
                                                 hipMemcpyHostToDevice, s), "copy"))
            return TR_ERR_HIP;
    }
    launch_eig_final(B, nblocks, su.d_inst, su.d_blocks, d_es, s);
    launch_recast_output(ddesc, B, kGrid, kP, phi, s);
    EigState* rs = (EigState*)h;
    if (!c->hip_ok(hipMemcpyAsync(rs, d_es, sizeof(EigState) * B, hipMemcpyDeviceToHost, s),
                   "copy"))
        return TR_ERR_HIP;
    const tr_status st = finish(c, "no_eigen output");
    if (st != TR_OK) return st;
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    tr_status worst = TR_OK;
    for (int i = 0; i < B; ++i) {
        const EigState& E = rs[i];
        const tr_status si = E.status == 0 ? TR_OK
                             : E.status == -4 ? TR_ERR_NONFINITE : TR_NOT_CONVERGED;
        if (si == TR_ERR_NONFINITE) c->fail("problem %d: non-finite iterate", i);
        if (stats) {
            tr_eigen_stats& o = stats[i];
            o.status = si;
            o.outer = E.outer;
            o.inner = variant == NO_EIGEN_CP ? E.outer : 0;
            o.k = E.k;
            o.dk = E.dk;
            o.dphi = E.dphi;
            o.balance_rel = NAN;
            o.seconds = secs;
        }
        if (si < 0 && (worst >= 0 || si < worst)) worst = si;
        else if (worst >= 0 && si > worst) worst = si;
    }
    return worst;
}
