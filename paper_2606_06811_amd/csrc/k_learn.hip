// k_learn.hip -- the learned cost model on gfx950: per-HSP features, and the
// 16-64-64-64-4 MLP (BF16 MFMA forward for inference and training, backward,
// Adam on FP32 master weights).
//
// The paper motivates predicting extension cost (Sec. 8: the work of an
// anchor-half is unknown until it has run; Sec. 9: sorting work up front as
// future load balancing) without defining a model, so the model is this
// library's own:
//   parameters, row-major (out x in): W1 64x16, b1 64, W2 64x64, b2 64,
//     W3 64x64, b3 64, W4 4x64, b4 4 (9668 floats);
//   forward: parameters and inputs rounded to BF16 (nearest, ties to even);
//     hidden layers A = bf16(relu(X W^T + b)) with FP32 accumulation; the
//     output layer is linear and stays FP32;
//   loss: mean of (Y - T)^2 over the batch and the 4 outputs;
//   backward: dY = 2 (Y - T) / (4 B) and every back-propagated signal
//     dZ = dA * [A > 0] are rounded to BF16 before they meet a product;
//     weight gradients G^T A_prev and bias gradients column sums of G, FP32;
//   Adam (0.9, 0.999, 1e-8) on the FP32 master weights, IEEE single ops in a
//     fixed order.
//
// Products run on the matrix cores: v_mfma_f32_16x16x16_bf16 computes a
// 16x16 FP32 tile D = A B + C.  Lane l supplies A[l % 16][4 (l / 16) + i] and
// B[4 (l / 16) + i][l % 16] (i = 0..3) and receives D[4 (l / 16) + i][l % 16].
#include "sfe_kernels.h"

namespace sfe {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define P_W1 0
#define P_B1 1024
#define P_W2 1088
#define P_B2 5184
#define P_W3 5248
#define P_B3 9344
#define P_W4 9408
#define P_B4 9664
#define P_N 9668
static_assert(P_N == SFE_MLP_NPARAMS, "parameter layout");

#define ALD 72                    // row stride (bf16) of 64-wide activation tiles in LDS
#define XLD 24                    // row stride (bf16) of 16-wide tiles in LDS

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x4 ld4(const uint16_t *p) { return *(const bf16x4 *)p; }
__device__ __forceinline__ bf16x4 pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
    bf16x4 v;
    v[0] = (short)a;
    v[1] = (short)b;
    v[2] = (short)c;
    v[3] = (short)d;
    return v;
}

// BF16 copy of the master weights.
__global__ void k_mlp_round(const float *__restrict__ master, uint16_t *__restrict__ p16) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P_N) p16[i] = to_bf16(master[i]);
}

// One hidden layer for the wave's 16 rows: dst = bf16(relu(src W^T + b)),
// src rows [16][IN] at stride sld, dst rows [16][64] at stride ALD.
template <int IN>
__device__ __forceinline__ void hidden_layer(const uint16_t *src, int sld, const uint16_t *__restrict__ W,
                                             const uint16_t *__restrict__ b, uint16_t *dst, int lane) {
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        const float bias = from_bf16(b[nt * 16 + r]);
        f32x4 acc = {bias, bias, bias, bias};
#pragma unroll
        for (int kt = 0; kt < IN / 16; kt++)
            acc = mfma(ld4(src + r * sld + kt * 16 + 4 * q), ld4(W + (nt * 16 + r) * IN + kt * 16 + 4 * q), acc);
#pragma unroll
        for (int i = 0; i < 4; i++) dst[(4 * q + i) * ALD + nt * 16 + r] = to_bf16(fmaxf(acc[i], 0.0f));
    }
}

// Output layer for the wave's 16 rows: lane l (l % 16 < 4) gets Y[4 (l / 16) + i][l % 16].
__device__ __forceinline__ f32x4 output_layer(const uint16_t *src, const uint16_t *__restrict__ P, int lane) {
    const int r = lane & 15, q = lane >> 4;
    const float bias = r < 4 ? from_bf16(P[P_B4 + r]) : 0.0f;
    f32x4 acc = {bias, bias, bias, bias};
#pragma unroll
    for (int kt = 0; kt < 4; kt++) {
        const bf16x4 w = r < 4 ? ld4(P + P_W4 + r * 64 + kt * 16 + 4 * q) : pack4(0, 0, 0, 0);
        acc = mfma(ld4(src + r * ALD + kt * 16 + 4 * q), w, acc);
    }
    return acc;
}

// Inference: Y[n x 4] from X[n x 16].  Each block takes 64 rows per pass, one
// wave per 16; the pass loop is uniform over the block.
__global__ void __launch_bounds__(256) k_mlp_forward(const float *__restrict__ X, int64_t n,
                                                     const uint16_t *__restrict__ P, float *__restrict__ Y) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[4][16 * XLD];
    __shared__ __attribute__((aligned(16))) uint16_t act[2][4][16 * ALD];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, q = lane >> 4;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
        const int64_t row = base + w * 16 + r;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row < n) x = *(const float4 *)(X + row * 16 + 4 * q);
        uint16_t *xr = &xs[w][r * XLD + 4 * q];
        xr[0] = to_bf16(x.x);
        xr[1] = to_bf16(x.y);
        xr[2] = to_bf16(x.z);
        xr[3] = to_bf16(x.w);
        __syncthreads();
        hidden_layer<16>(xs[w], XLD, P + P_W1, P + P_B1, act[0][w], lane);
        __syncthreads();
        hidden_layer<64>(act[0][w], ALD, P + P_W2, P + P_B2, act[1][w], lane);
        __syncthreads();
        hidden_layer<64>(act[1][w], ALD, P + P_W3, P + P_B3, act[0][w], lane);
        __syncthreads();
        const f32x4 y = output_layer(act[0][w], P, lane);
        if (r < 4) {
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int64_t rr = base + w * 16 + 4 * q + i;
                if (rr < n) Y[rr * 4 + r] = y[i];
            }
        }
        __syncthreads();
    }
}

// Weight gradient tile: out rows [16 mt, 16 mt + 16) x in columns [16 nt, ..)
// of G^T A over the block's 64 samples.  G [64][gld] (column = output unit),
// A [64][ald] (column = input unit).
__device__ __forceinline__ f32x4 wgrad_tile(const uint16_t *G, int gld, int mt, const uint16_t *A, int ald, int nt,
                                            int lane) {
    const int r = lane & 15, q = lane >> 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; kt++) {
        const int s = kt * 16 + 4 * q;
        const bf16x4 a = pack4(G[(s + 0) * gld + mt * 16 + r], G[(s + 1) * gld + mt * 16 + r],
                               G[(s + 2) * gld + mt * 16 + r], G[(s + 3) * gld + mt * 16 + r]);
        const bf16x4 b = pack4(A[(s + 0) * ald + nt * 16 + r], A[(s + 1) * ald + nt * 16 + r],
                               A[(s + 2) * ald + nt * 16 + r], A[(s + 3) * ald + nt * 16 + r]);
        acc = mfma(a, b, acc);
    }
    return acc;
}

// Back-propagated signal of a hidden layer for the wave's 16 rows:
// Gout = bf16((Gin W) * [Aprev > 0]); Gin [16][gld] with KO output units,
// W (KO x 64, bf16 global), Aprev and Gout [16][ALD].
template <int KO>
__device__ __forceinline__ void back_layer(const uint16_t *Gin, int gld, const uint16_t *__restrict__ W,
                                           const uint16_t *Aprev, uint16_t *Gout, int lane) {
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < (KO + 15) / 16; kt++) {
            const int o = kt * 16 + 4 * q;
            uint16_t w[4];
#pragma unroll
            for (int i = 0; i < 4; i++) w[i] = (o + i < KO) ? W[(o + i) * 64 + nt * 16 + r] : (uint16_t)0;
            acc = mfma(ld4(Gin + r * gld + kt * 16 + 4 * q), pack4(w[0], w[1], w[2], w[3]), acc);
        }
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int s = 4 * q + i, c = nt * 16 + r;
            const bool on = from_bf16(Aprev[s * ALD + c]) > 0.0f;
            Gout[s * ALD + c] = on ? to_bf16(acc[i]) : (uint16_t)0;
        }
    }
}

// Gradient of one batch: block b takes batch samples [64 b, 64 b + 64) (ids of
// X/T rows), writes its parameter-gradient partial part[b][P_N] and its sum
// of squared errors sse[b].  B is the batch size (the scale of dY).
__global__ void __launch_bounds__(256) k_mlp_grad(const float *__restrict__ X, const float *__restrict__ T,
                                                  const int32_t *__restrict__ ids, int32_t B,
                                                  const uint16_t *__restrict__ P, float *__restrict__ part,
                                                  float *__restrict__ sse) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[64 * XLD];
    __shared__ __attribute__((aligned(16))) uint16_t a1[64 * ALD], a2[64 * ALD], a3[64 * ALD];
    __shared__ __attribute__((aligned(16))) uint16_t ga[64 * ALD], gb[64 * ALD];
    __shared__ __attribute__((aligned(16))) uint16_t g4[64 * XLD];
    __shared__ float red[256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 15, q = lane >> 4;
    const int s0 = blockIdx.x * 64;
    float *out = part + (size_t)blockIdx.x * P_N;
    {   // inputs (rows past the batch are zero and carry no gradient)
        const int s = tid >> 2, k = (tid & 3) * 4;
        float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
        if (s0 + s < B) x = *(const float4 *)(X + (int64_t)ids[s0 + s] * 16 + k);
        xs[s * XLD + k + 0] = to_bf16(x.x);
        xs[s * XLD + k + 1] = to_bf16(x.y);
        xs[s * XLD + k + 2] = to_bf16(x.z);
        xs[s * XLD + k + 3] = to_bf16(x.w);
        for (int c = tid; c < 64 * XLD; c += 256) g4[c] = 0;
    }
    __syncthreads();
    const int rw = w * 16;      // the wave's rows
    hidden_layer<16>(xs + rw * XLD, XLD, P + P_W1, P + P_B1, a1 + rw * ALD, lane);
    __syncthreads();
    hidden_layer<64>(a1 + rw * ALD, ALD, P + P_W2, P + P_B2, a2 + rw * ALD, lane);
    __syncthreads();
    hidden_layer<64>(a2 + rw * ALD, ALD, P + P_W3, P + P_B3, a3 + rw * ALD, lane);
    __syncthreads();
    float my_sse = 0.0f;
    {
        const f32x4 y = output_layer(a3 + rw * ALD, P, lane);
        if (r < 4) {
            const float scale = (float)(4 * B);
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int s = rw + 4 * q + i;
                if (s0 + s < B) {
                    const float d = __fsub_rn(y[i], T[(int64_t)ids[s0 + s] * 4 + r]);
                    my_sse = __fmaf_rn(d, d, my_sse);
                    g4[s * XLD + r] = to_bf16(__fdiv_rn(__fmul_rn(2.0f, d), scale));
                }
            }
        }
    }
    red[tid] = my_sse;
    __syncthreads();
    // layer 4: dW4 (4 x 64), db4, and the signal into layer 3
    {
        const f32x4 acc = wgrad_tile(g4, XLD, 0, a3, ALD, w, lane);
        if (q == 0) {
#pragma unroll
            for (int i = 0; i < 4; i++) out[P_W4 + i * 64 + w * 16 + r] = acc[i];
        }
        if (tid < 4) {
            float sb = 0.0f;
            for (int s = 0; s < 64; s++) sb = __fadd_rn(sb, from_bf16(g4[s * XLD + tid]));
            out[P_B4 + tid] = sb;
        }
        back_layer<4>(g4 + rw * XLD, XLD, P + P_W4, a3 + rw * ALD, ga + rw * ALD, lane);
    }
    __syncthreads();
    // layer 3: dW3 = G3^T A2, db3, G2
    {
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            const f32x4 acc = wgrad_tile(ga, ALD, w, a2, ALD, nt, lane);
#pragma unroll
            for (int i = 0; i < 4; i++) out[P_W3 + (w * 16 + 4 * q + i) * 64 + nt * 16 + r] = acc[i];
        }
        if (tid < 64) {
            float sb = 0.0f;
            for (int s = 0; s < 64; s++) sb = __fadd_rn(sb, from_bf16(ga[s * ALD + tid]));
            out[P_B3 + tid] = sb;
        }
        back_layer<64>(ga + rw * ALD, ALD, P + P_W3, a2 + rw * ALD, gb + rw * ALD, lane);
    }
    __syncthreads();
    // layer 2: dW2 = G2^T A1, db2, G1
    {
#pragma unroll
        for (int nt = 0; nt < 4; nt++) {
            const f32x4 acc = wgrad_tile(gb, ALD, w, a1, ALD, nt, lane);
#pragma unroll
            for (int i = 0; i < 4; i++) out[P_W2 + (w * 16 + 4 * q + i) * 64 + nt * 16 + r] = acc[i];
        }
        if (tid < 64) {
            float sb = 0.0f;
            for (int s = 0; s < 64; s++) sb = __fadd_rn(sb, from_bf16(gb[s * ALD + tid]));
            out[P_B2 + tid] = sb;
        }
        back_layer<64>(gb + rw * ALD, ALD, P + P_W2, a1 + rw * ALD, ga + rw * ALD, lane);
    }
    __syncthreads();
    // layer 1: dW1 = G1^T X, db1
    {
        const f32x4 acc = wgrad_tile(ga, ALD, w, xs, XLD, 0, lane);
#pragma unroll
        for (int i = 0; i < 4; i++) out[P_W1 + (w * 16 + 4 * q + i) * 16 + r] = acc[i];
        if (tid < 64) {
            float sb = 0.0f;
            for (int s = 0; s < 64; s++) sb = __fadd_rn(sb, from_bf16(ga[s * ALD + tid]));
            out[P_B1 + tid] = sb;
        }
    }
    if (tid == 0) {
        float t = 0.0f;
        for (int i = 0; i < 256; i++) t = __fadd_rn(t, red[i]);
        sse[blockIdx.x] = t;
    }
}

// Sums the nb block partials (in block order) and either stores the gradient
// (grad != null) or applies one Adam step to the master weights and refreshes
// their BF16 copy.  c1 = 1 - beta1^t, c2 = 1 - beta2^t.  Block 0 also writes
// the batch loss sum(sse) / (4 B) to *loss when loss is not null.
__global__ void k_mlp_apply(const float *__restrict__ part, int nb, const float *__restrict__ sse, int32_t B,
                            float *__restrict__ grad, float *__restrict__ master, float *__restrict__ m,
                            float *__restrict__ v, uint16_t *__restrict__ p16, float lr, float c1, float c2,
                            float *__restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (loss && p == 0) {
        float t = 0.0f;
        for (int b = 0; b < nb; b++) t = __fadd_rn(t, sse[b]);
        *loss = __fdiv_rn(t, (float)(4 * B));
    }
    if (p >= P_N) return;
    float g = 0.0f;
    for (int b = 0; b < nb; b++) g = __fadd_rn(g, part[(size_t)b * P_N + p]);
    if (grad) {
        grad[p] = g;
        return;
    }
    const float mm = __fadd_rn(__fmul_rn(0.9f, m[p]), __fmul_rn(0.1f, g));
    const float vv = __fadd_rn(__fmul_rn(0.999f, v[p]), __fmul_rn(__fmul_rn(0.001f, g), g));
    const float mh = __fdiv_rn(mm, c1), vh = __fdiv_rn(vv, c2);
    const float pp = __fsub_rn(master[p], __fdiv_rn(__fmul_rn(lr, mh), __fadd_rn(__fsqrt_rn(vh), 1e-8f)));
    m[p] = mm;
    v[p] = vv;
    master[p] = pp;
    p16[p] = to_bf16(pp);
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------
// Counts over positions [lo, hi) of one packed set (absolute positions):
// C/G bases, N bases, soft-masked bases.
__device__ void window_counts(const SeqSetView &S, int64_t lo, int64_t hi, int *gc, int *nn, int *soft) {
    int g = 0, n = 0, sm = 0;
    for (int64_t p = lo; p < hi;) {
        if ((p & 31) == 0 && p + 32 <= hi) {
            const uint32_t w0 = S.bases[p >> 4], w1 = S.bases[(p >> 4) + 1];
            g += __popc((w0 ^ (w0 >> 1)) & 0x55555555u) + __popc((w1 ^ (w1 >> 1)) & 0x55555555u);
            const uint32_t nb = S.nbits[p >> 5];
            // an N is stored as code 0 and so never counts as C/G
            n += __popc(nb);
            sm += __popc(S.sbits[p >> 5]);
            p += 32;
        } else {
            const uint32_t w = S.bases[p >> 4];
            const int c = (int)((w >> ((p & 15) * 2)) & 3u);
            const bool isn = (S.nbits[p >> 5] >> (p & 31)) & 1u;
            n += isn;
            g += (!isn && (c == 1 || c == 2));
            sm += (S.sbits[p >> 5] >> (p & 31)) & 1u;
            p++;
        }
    }
    *gc = g;
    *nn = n;
    *soft = sm;
}

// One thread per HSP.  order/okey: HSP ids sorted by (unit, anchor t) and
// their anchor t; ustart/uend: the sorted range of each unit.
__global__ void k_hsp_features(const sfe_hsp *__restrict__ h, int64_t n, const int32_t *__restrict__ unit_of,
                               const UnitDesc *__restrict__ units, SeqSetView T, int64_t nt, SeqSetView Qp,
                               SeqSetView Qm, const uint32_t *__restrict__ order, const uint32_t *__restrict__ okey,
                               const int64_t *__restrict__ ustart, const int64_t *__restrict__ uend,
                               float *__restrict__ F) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const sfe_hsp H = h[x];
    const int32_t u = unit_of[2 * H.query_id + H.strand];
    const UnitDesc U = units[u];
    const SeqSetView Q = U.strand ? Qm : Qp;
    const int64_t L = H.len;
    int match = 0, ts = 0, tv = 0;
    for (int64_t k = 0; k < L; k++) {
        const int a = base_code(T, (int64_t)H.t0 + k), b = base_code(Q, U.seq_start + H.q0 + k);
        if (a == b && a < 4) match++;
        else if (a < 4 && b < 4 && (a ^ b) == 2) ts++;
        else tv++;
    }
    const int64_t ta = (int64_t)H.t0 + (L - 1) / 2, qa = (int64_t)H.q0 + (L - 1) / 2;
    const int64_t dg = ta - qa;
    int near = 0, wide = 0;
    int64_t down = -1, up = -1;
    {
        // first sorted position with anchor >= ta - 10000 inside the unit
        int64_t lo = ustart[u], hi = uend[u];
        const int64_t want = ta - 10000;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)okey[mid] < want) lo = mid + 1;
            else hi = mid;
        }
        for (int64_t y = lo; y < uend[u] && (int64_t)okey[y] <= ta + 10000; y++) {
            const uint32_t id = order[y];
            if ((int64_t)id == x) continue;
            const sfe_hsp G = h[id];
            const int64_t tb = (int64_t)G.t0 + ((int64_t)G.len - 1) / 2, qb = (int64_t)G.q0 + ((int64_t)G.len - 1) / 2;
            const int64_t dt = tb - ta;
            wide++;
            const int64_t dd = (tb - qb) - dg;
            if (dd <= 64 && dd >= -64) {
                if (dt <= 5000 && dt >= -5000) near++;
                if (dt > 0 && (down < 0 || dt < down)) down = dt;
                if (dt < 0 && (up < 0 || -dt < up)) up = -dt;
            }
        }
    }
    int tg, tn, tsm, qg, qn, qsm;
    const int64_t tlo = max((int64_t)0, ta - 1000), thi = min(nt, ta + 1000);
    const int64_t qlo = max((int64_t)0, qa - 1000), qhi = min(U.len, qa + 1000);
    window_counts(T, tlo, thi, &tg, &tn, &tsm);
    window_counts(Q, U.seq_start + qlo, U.seq_start + qhi, &qg, &qn, &qsm);
    const float Lf = (float)L;
    float *f = F + x * 16;
    f[0] = (float)H.score / 4096.0f;
    f[1] = log2f(1.0f + Lf) / 16.0f;
    f[2] = (float)match / Lf;
    f[3] = (float)ts / Lf;
    f[4] = (float)tv / Lf;
    f[5] = (float)((int64_t)H.t0 - (int64_t)H.q0) / (float)nt;
    f[6] = (float)H.strand;
    f[7] = (float)ta / (float)nt;
    f[8] = (float)qa / (float)U.len;
    const int tnn = (int)(thi - tlo) - tn, qnn = (int)(qhi - qlo) - qn;
    f[9] = tnn > 0 ? (float)tg / (float)tnn : 0.0f;
    f[10] = qnn > 0 ? (float)qg / (float)qnn : 0.0f;
    f[11] = log2f(1.0f + (float)near) / 8.0f;
    f[12] = log2f(1.0f + (float)wide) / 8.0f;
    f[13] = down > 0 ? log2f(1.0f + (float)down) / 16.0f : 1.0f;
    f[14] = up > 0 ? log2f(1.0f + (float)up) / 16.0f : 1.0f;
    f[15] = thi > tlo ? (float)tsm / (float)(thi - tlo) : 0.0f;
}

// Sort keys (unit << 32 | anchor t) and ids of the HSPs.
__global__ void k_hsp_anchor_keys(const sfe_hsp *__restrict__ h, int64_t n, const int32_t *__restrict__ unit_of,
                                  uint64_t *__restrict__ key, uint32_t *__restrict__ ids) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const sfe_hsp H = h[x];
    key[x] = ((uint64_t)(uint32_t)unit_of[2 * H.query_id + H.strand] << 32) | (uint64_t)(H.t0 + (H.len - 1) / 2);
    ids[x] = (uint32_t)x;
}

// After the (unit, anchor) sort: okey[y] = anchor t of order[y], and the
// range [ustart[u], uend[u]) of each unit (units absent keep 0, 0).
__global__ void k_hsp_unit_ranges(const sfe_hsp *__restrict__ h, const int32_t *__restrict__ unit_of,
                                  const uint32_t *__restrict__ order, int64_t n, uint32_t *__restrict__ okey,
                                  int64_t *__restrict__ ustart, int64_t *__restrict__ uend) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    const sfe_hsp H = h[order[y]];
    okey[y] = H.t0 + (H.len - 1) / 2;
    const int32_t u = unit_of[2 * H.query_id + H.strand];
    if (y == 0 || unit_of[2 * h[order[y - 1]].query_id + h[order[y - 1]].strand] != u) ustart[u] = y;
    if (y == n - 1 || unit_of[2 * h[order[y + 1]].query_id + h[order[y + 1]].strand] != u) uend[u] = y + 1;
}

void launch_mlp_round(const float *master, uint16_t *p16, hipStream_t st) {
    k_mlp_round<<<(P_N + 255) / 256, 256, 0, st>>>(master, p16);
}
void launch_mlp_forward(const float *X, int64_t n, const uint16_t *p16, float *Y, hipStream_t st) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 63) / 64, 4096);
    k_mlp_forward<<<(unsigned)blocks, 256, 0, st>>>(X, n, p16, Y);
}
void launch_mlp_grad(const float *X, const float *T, const int32_t *ids, int32_t B, const uint16_t *p16,
                     float *part, float *sse, hipStream_t st) {
    if (B <= 0) return;
    k_mlp_grad<<<(unsigned)((B + 63) / 64), 256, 0, st>>>(X, T, ids, B, p16, part, sse);
}
void launch_mlp_apply(const float *part, int nb, const float *sse, int32_t B, float *grad, float *master, float *m,
                      float *v, uint16_t *p16, float lr, float c1, float c2, float *loss, hipStream_t st) {
    k_mlp_apply<<<(P_N + 255) / 256, 256, 0, st>>>(part, nb, sse, B, grad, master, m, v, p16, lr, c1, c2, loss);
}
void launch_hsp_features(const sfe_hsp *h, int64_t n, const int32_t *unit_of, const UnitDesc *units, SeqSetView T,
                         int64_t nt, SeqSetView Qp, SeqSetView Qm, const uint32_t *order, const uint32_t *okey,
                         const int64_t *ustart, const int64_t *uend, float *F, hipStream_t st) {
    if (n <= 0) return;
    k_hsp_features<<<(unsigned)((n + 127) / 128), 128, 0, st>>>(h, n, unit_of, units, T, nt, Qp, Qm, order, okey,
                                                                  ustart, uend, F);
}
void launch_hsp_anchor_keys(const sfe_hsp *h, int64_t n, const int32_t *unit_of, uint64_t *key, uint32_t *ids,
                            hipStream_t st) {
    if (n <= 0) return;
    k_hsp_anchor_keys<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(h, n, unit_of, key, ids);
}
void launch_hsp_unit_ranges(const sfe_hsp *h, const int32_t *unit_of, const uint32_t *order, int64_t n,
                            uint32_t *okey, int64_t *ustart, int64_t *uend, hipStream_t st) {
    if (n <= 0) return;
    k_hsp_unit_ranges<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(h, unit_of, order, n, okey, ustart, uend);
}

}  // namespace sfe
