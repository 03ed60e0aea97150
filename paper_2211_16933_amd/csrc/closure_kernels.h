// Device kernels of the learned closure (gfx950): the MLP 12 -> 64 -> 64 -> 64 -> Q_s with
// SiLU on bfloat16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), its
// backward pass and Adam, and the per-cell closure: moments of every row, the 12 inputs,
// the correction added to the student's L[phi], and the training samples.  Included by
// elb.hip only.  The parameter layout and the normalisation block are those of
// mlp_device.h.  The stage kernel carries a fused form of k_closure_rows and
// k_closure_apply (elb_set_closure with enabled = 1); these two kernels are the separate
// form (enabled = 2).
#pragma once
#include <hip/hip_runtime.h>

#include "elb_kernels.h"
#include "mlp_device.h"

namespace elb {

// acc[t] (t < NT) = A[16][K] x B^T for the 16-column block t of B, where A is a bf16 tile
// with row stride as and B is [N][K] bf16 with row stride bs (both in LDS).  Operand lane
// layout of v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16], i < 8; the result D[4 (l / 16) + r][l % 16] sits in acc[r].
template <int K, int NT>
__device__ inline void mma_rows16(const unsigned short *A, int as, const unsigned short *B, int bs,
                                  floatx4 acc[NT], int lane)
{
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int r = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll
    for (int kk = 0; kk < K / 32; ++kk) {
        bf16x8 a = ld8(A + r * as + kk * 32 + kq);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bf16x8 b = ld8(B + (t * 16 + r) * bs + kk * 32 + kq);
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
}

// Weights of the forward pass in LDS (bf16) and the biases (FP32).
struct alignas(16) MlpSmem {
    unsigned short w1[MLP_H * WS1];
    unsigned short w2[MLP_H * WSH];
    unsigned short w3[MLP_H * WSH];
    unsigned short w4[MLP_OUT * WSH];
    float bias[3 * MLP_H + MLP_OUT];
    unsigned short act[4][2][16 * AS];   // per wave: two activation tiles (ping-pong)
};

__device__ inline void mlp_stage_weights(MlpSmem &s, const unsigned short *wb, const float *params)
{
    for (int j = threadIdx.x; j < MLP_H * MLP_K1; j += blockDim.x)
        s.w1[(j / MLP_K1) * WS1 + j % MLP_K1] = wb[OFF_W1 + j];
    for (int j = threadIdx.x; j < MLP_H * MLP_H; j += blockDim.x) {
        s.w2[(j / MLP_H) * WSH + j % MLP_H] = wb[OFF_W2 + j];
        s.w3[(j / MLP_H) * WSH + j % MLP_H] = wb[OFF_W3 + j];
    }
    for (int j = threadIdx.x; j < MLP_OUT * MLP_H; j += blockDim.x)
        s.w4[(j / MLP_H) * WSH + j % MLP_H] = wb[OFF_W4 + j];
    for (int j = threadIdx.x; j < MLP_H; j += blockDim.x) {
        s.bias[j] = params[OFF_B1 + j];
        s.bias[MLP_H + j] = params[OFF_B2 + j];
        s.bias[2 * MLP_H + j] = params[OFF_B3 + j];
    }
    for (int j = threadIdx.x; j < MLP_OUT; j += blockDim.x) s.bias[3 * MLP_H + j] = params[OFF_B4 + j];
}

// Forward pass of the 16 rows whose bf16 inputs are in s.act[wave][0] (columns 0..31).
// Pre-activations of the hidden layers go to z (row stride 64, 3 layers of zstride floats)
// when z != NULL, for rows < nvalid.  Output y[16][16] (FP32) in the D layout of acc4.
// Every wave of the block must call this (it synchronises the block between layers).
__device__ inline void mlp_forward_rows(MlpSmem &s, int wave, int lane, float *z, size_t zstride,
                                        int nvalid, floatx4 &acc4)
{
    unsigned short *a0 = s.act[wave][0], *a1 = s.act[wave][1];
    floatx4 acc[4];
    const int col = lane & 15, rq = 4 * (lane >> 4);
    // layer 1: K = 32
    mma_rows16<MLP_K1, 4>(a0, AS, s.w1, WS1, acc, lane);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rq + r, c = t * 16 + col;
            float zz = acc[t][r] + s.bias[c];
            if (z && row < nvalid) z[(size_t)row * MLP_H + c] = zz;
            a1[row * AS + c] = f2bf(silu(zz));
        }
    __syncthreads();
    // layers 2 and 3: K = 64
#pragma unroll
    for (int l = 0; l < 2; ++l) {
        const unsigned short *ain = l == 0 ? a1 : a0;
        unsigned short *aout = l == 0 ? a0 : a1;
        mma_rows16<MLP_H, 4>(ain, AS, l == 0 ? s.w2 : s.w3, WSH, acc, lane);
        __syncthreads();  // every lane has read ain / may overwrite aout (aliases a0 at l = 0)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rq + r, c = t * 16 + col;
                float zz = acc[t][r] + s.bias[(l + 1) * MLP_H + c];
                if (z && row < nvalid) z[(l + 1) * zstride + (size_t)row * MLP_H + c] = zz;
                aout[row * AS + c] = f2bf(silu(zz));
            }
        __syncthreads();
    }
    // layer 4: 16 outputs
    floatx4 o[1];
    mma_rows16<MLP_H, 1>(a1, AS, s.w4, WSH, o, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) o[0][r] += s.bias[3 * MLP_H + col];
    acc4 = o[0];
}

// --------------------------------------------------------------------------------------
// Training forward: rows b < batch of x[index[b]] (or x[b]), normalised, through the MLP.
// y [batch][16] (normalised outputs); a0 [batch][32] bf16 inputs and z [3][batch][64]
// pre-activations are kept for the backward pass.
// --------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_forward(const unsigned short *wb, const float *params,
                                                     const float *norm, const float *x,
                                                     const int *index, int batch, float *y,
                                                     unsigned short *a0_out, float *z)
{
    __shared__ MlpSmem s;
    mlp_stage_weights(s, wb, params);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row0 = blockIdx.x * MLP_ROWS + wave * 16;
    // inputs: lane l fills row l % 16, columns 8 (l / 16) .. + 7
    {
        const int r = lane & 15, c0 = 8 * (lane >> 4);
        const int b = row0 + r;
        for (int c = c0; c < c0 + 8; ++c) {
            float v = 0.f;
            if (b < batch && c < MLP_IN) {
                const int src = index ? index[b] : b;
                v = (x[(size_t)src * MLP_IN + c] - norm[NRM_IN_MEAN + c]) / norm[NRM_IN_STD + c];
            }
            unsigned short h = f2bf(v);
            s.act[wave][0][r * AS + c] = h;
            if (b < batch) a0_out[(size_t)b * MLP_K1 + c] = h;
        }
    }
    __syncthreads();
    const int nvalid = batch - row0;
    floatx4 o;
    mlp_forward_rows(s, wave, lane, row0 < batch ? z + (size_t)row0 * MLP_H : nullptr,
                     (size_t)batch * MLP_H, nvalid, o);
    const int col = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (rq + r < nvalid) y[(size_t)(row0 + rq + r) * MLP_OUT + col] = o[r];
}

// Loss mean((y - t_norm)^2) over batch x q_out and its gradient dy (zero on padded outputs);
// t_norm = (t[index[b]] - out_mean) / out_std.  Per-block partial sums of the loss go to
// part[blockIdx.x] (summed by k_sum_partials).
__global__ __launch_bounds__(256) void k_mlp_loss(const float *y, const float *t, const int *index,
                                                  const float *norm, int batch, int q_out, float *dy,
                                                  double *part)
{
    __shared__ double red[256];
    double acc = 0.0;
    const double scale = 2.0 / ((double)batch * q_out);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < batch * MLP_OUT; j += gridDim.x * blockDim.x) {
        const int b = j / MLP_OUT, o = j - b * MLP_OUT;
        float g = 0.f;
        if (o < q_out) {
            const int src = index ? index[b] : b;
            float tn = (t[(size_t)src * q_out + o] - norm[NRM_OUT_MEAN + o]) / norm[NRM_OUT_STD + o];
            float d = y[j] - tn;
            acc += (double)d * d;
            g = (float)(scale * d);
        }
        dy[j] = g;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_partials(const double *part, int n, double scale, double *out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s * scale;
    }
}

// --------------------------------------------------------------------------------------
// Backward pass, per row: dz4 = dy; da_l = bf16(dz_{l+1}) W_{l+1}; dz_l = da_l SiLU'(z_l).
// dz [3][batch][64] (layers 1..3).  Transposed weights in LDS: W4^T [64][32] (outputs
// 16..31 zero), W3^T, W2^T [64][64].
// --------------------------------------------------------------------------------------
struct alignas(16) BwdSmem {
    unsigned short w4t[MLP_H * WS1];
    unsigned short w3t[MLP_H * WSH];
    unsigned short w2t[MLP_H * WSH];
    unsigned short act[4][16 * AS];
};

__global__ __launch_bounds__(256) void k_mlp_backward(const unsigned short *wb, const float *dy,
                                                      const float *z, int batch, float *dz)
{
    __shared__ BwdSmem s;
    for (int j = threadIdx.x; j < MLP_H * MLP_K1; j += blockDim.x) {
        const int n = j / MLP_K1, k = j % MLP_K1;   // W4^T[n][k] = W4[k][n]
        s.w4t[n * WS1 + k] = k < MLP_OUT ? wb[OFF_W4 + k * MLP_H + n] : (unsigned short)0;
    }
    for (int j = threadIdx.x; j < MLP_H * MLP_H; j += blockDim.x) {
        const int n = j / MLP_H, k = j % MLP_H;
        s.w3t[n * WSH + k] = wb[OFF_W3 + k * MLP_H + n];
        s.w2t[n * WSH + k] = wb[OFF_W2 + k * MLP_H + n];
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int row0 = blockIdx.x * MLP_ROWS + wave * 16;
    const int nvalid = batch - row0;
    unsigned short *A = s.act[wave];
    {
        const int r = lane & 15, c0 = 8 * (lane >> 4);
        for (int c = c0; c < c0 + 8; ++c) {
            float v = (c < MLP_OUT && r < nvalid) ? dy[(size_t)(row0 + r) * MLP_OUT + c] : 0.f;
            A[r * AS + c] = f2bf(v);
        }
    }
    __syncthreads();
    const int col = lane & 15, rq = 4 * (lane >> 4);
    floatx4 acc[4];
    const size_t lstride = (size_t)batch * MLP_H;
#pragma unroll
    for (int l = 2; l >= 0; --l) {  // hidden layer l + 1
        if (l == 2) mma_rows16<MLP_K1, 4>(A, AS, s.w4t, WS1, acc, lane);
        else mma_rows16<MLP_H, 4>(A, AS, l == 1 ? s.w3t : s.w2t, WSH, acc, lane);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rq + r, c = t * 16 + col;
                float d = 0.f;
                if (row < nvalid) {
                    const size_t o = l * lstride + (size_t)(row0 + row) * MLP_H + c;
                    d = acc[t][r] * dsilu(z[o]);
                    dz[o] = d;
                }
                A[row * AS + c] = f2bf(d);
            }
        __syncthreads();
    }
}

// Weight gradients over a chunk of WGRAD_ROWS batch rows: partial dW_l = bf16(dz_l)^T a_{l-1}
// and db_l = sum dz_l, written to part[blockIdx.x][MLP_PARAMS].  a_0 is the stored bf16
// input, a_l = bf16(SiLU(z_l)).
struct alignas(16) WgradSmem {
    unsigned short gt[MLP_H * GS_T];   // dz^T [out][rows]
    unsigned short at[MLP_H * GS_T];   // a^T  [in][rows]
    float gf[WGRAD_ROWS * MLP_H];      // dz in FP32 [rows][out] (bias gradients)
};

__global__ __launch_bounds__(256) void k_mlp_wgrad(const float *dy, const float *dz, const float *z,
                                                   const unsigned short *a0, int batch, float *part)
{
    __shared__ WgradSmem s;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int b0 = blockIdx.x * WGRAD_ROWS;
    const int nrow = min(WGRAD_ROWS, batch - b0);
    float *P = part + (size_t)blockIdx.x * MLP_PARAMS;
    const size_t lstride = (size_t)batch * MLP_H;
    for (int layer = 4; layer >= 1; --layer) {
        const int nout = layer == 4 ? MLP_OUT : MLP_H;
        const int kin = layer == 1 ? MLP_K1 : MLP_H;
        const float *g = layer == 4 ? dy : dz + (size_t)(layer - 1) * lstride;
        __syncthreads();
        for (int j = threadIdx.x; j < WGRAD_ROWS * nout; j += blockDim.x) {
            const int b = j / nout, n = j - b * nout;
            float v = b < nrow ? g[(size_t)(b0 + b) * nout + n] : 0.f;
            s.gt[n * GS_T + b] = f2bf(v);
            s.gf[b * nout + n] = v;
        }
        for (int j = threadIdx.x; j < WGRAD_ROWS * kin; j += blockDim.x) {
            const int b = j / kin, k = j - b * kin;
            unsigned short v = 0;
            if (b < nrow) {
                if (layer == 1) v = a0[(size_t)(b0 + b) * MLP_K1 + k];
                else v = f2bf(silu(z[(size_t)(layer - 2) * lstride + (size_t)(b0 + b) * MLP_H + k]));
            }
            s.at[k * GS_T + b] = v;
        }
        __syncthreads();
        // bias gradient: plain FP32 sums in row order, from the staged copy
        const int boff = layer == 1 ? OFF_B1 : layer == 2 ? OFF_B2 : layer == 3 ? OFF_B3 : OFF_B4;
        for (int n = threadIdx.x; n < nout; n += blockDim.x) {
            float acc = 0.f;
            for (int b = 0; b < nrow; ++b) acc += s.gf[b * nout + n];
            P[boff + n] = acc;
        }
        const int woff = layer == 1 ? OFF_W1 : layer == 2 ? OFF_W2 : layer == 3 ? OFF_W3 : OFF_W4;
        const int tn = nout / 16, tk = kin / 16;
        for (int t = wave; t < tn * tk; t += 4) {
            const int tm = t / tk, tc = t - tm * tk;
            floatx4 acc[1];
            mma_rows16<WGRAD_ROWS, 1>(s.gt + tm * 16 * GS_T, GS_T, s.at + tc * 16 * GS_T, GS_T, acc, lane);
            const int c = tc * 16 + (lane & 15), rq = 4 * (lane >> 4);
#pragma unroll
            for (int r = 0; r < 4; ++r) P[woff + (tm * 16 + rq + r) * kin + c] = acc[0][r];
        }
    }
}

// grad[j] = sum over blocks of part[blk][j], in block order (deterministic)
__global__ void k_mlp_reduce(const float *part, int nblk, float *grad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= MLP_PARAMS) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * MLP_PARAMS + j];
    grad[j] = s;
}

// Adam (Kingma and Ba, 2015) on the FP32 master parameters; refreshes the bf16 copy.
__global__ void k_mlp_adam(float *w, unsigned short *wb, float *m, float *v, const float *g, int count,
                           float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    float gj = g[j];
    float mj = b1 * m[j] + (1.f - b1) * gj;
    float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    float wj = w[j] - lr * (mj / c1) / (sqrtf(vj / c2) + eps);
    w[j] = wj;
    wb[j] = f2bf(wj);
}

__global__ void k_round_bf16(const float *w, unsigned short *wb, int count)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) wb[j] = f2bf(w[j]);
}

// --------------------------------------------------------------------------------------
// Closure of a student context
// --------------------------------------------------------------------------------------
// (n, u, T, q, Pxx) of rows r < nx + 6 (cell r - 3; periodic problems wrap the cell index,
// others read the ghost rows).  Deviation storage adds ref; with U the density, velocity
// and temperature come from the conserved densities.
template <typename R>
__global__ void k_closure_rows(const R *psi, const double *ref, const double *U, const double *p,
                               int nx, int Q, int periodic, double *rows5)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nx + 2 * NG) return;
    const int sr = row_of(r - NG, nx, periodic);
    const R *ph = psi + (size_t)sr * 2 * Q;
    const R *th = ph + Q;
    double n = 0, j = 0, e2 = 0;
    for (int k = 0; k < Q; ++k) {
        double v = (double)ph[k] + ref[k];
        n += v;
        j += p[k] * v;
        e2 += 0.5 * (p[k] * p[k] * v + (double)th[k] + ref[Q + k]);
    }
    if (U) {
        const double *Ui = U + 3 * (size_t)sr;
        n = Ui[0];
        j = Ui[1];
        e2 = Ui[2];
    }
    double u = j / n, pxx = 0, e = 0, q = 0;
    for (int k = 0; k < Q; ++k) {
        double xi = p[k] - u;
        double vp = (double)ph[k] + ref[k], vt = (double)th[k] + ref[Q + k];
        double ek = 0.5 * xi * xi * vp + 0.5 * vt;
        pxx += xi * xi * vp;
        e += ek;
        q += xi * ek;
    }
    double T = U ? (2.0 * e2 / n - u * u) / 3.0 : e / (1.5 * n);
    double *o = rows5 + 5 * (size_t)r;
    o[0] = n; o[1] = u; o[2] = T; o[3] = q; o[4] = pxx;
}

struct ClosureConst {
    double dx, b, mu_ref, denseness, log10kn;
};

// The 12 inputs of cell i from the row moments, and n / tau.
__device__ inline void closure_features(const double *rows5, int i, const ClosureConst &cc,
                                        double x[MLP_IN], double *scale)
{
    const double *c = rows5 + 5 * (size_t)(i + NG);
    const double n = c[0], u = c[1], T = c[2], q = c[3], pxx = c[4];
    double d[5];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const double *m = rows5 + 5 * (size_t)i + f;  // row i = cell i - 3
        d[f] = (-m[0] + 9.0 * m[5] - 45.0 * m[10] + 45.0 * m[20] - 9.0 * m[25] + m[30]) / (60.0 * cc.dx);
    }
    const double eta = 0.25 * cc.b * n;
    const double chi = chi_set(eta);
    const double y = cc.b * n * chi;
    const double itau = inv_tau(cc.mu_ref, n, T, chi, y);
    const double sT = sqrt(T);
    const double lam = sT / itau;
    const double qs = n * T * sT;
    x[0] = n; x[1] = u; x[2] = T;
    x[3] = q / qs;
    x[4] = pxx / (n * T) - 1.0;
    x[5] = lam * d[0] / n;
    x[6] = lam * d[1] / sT;
    x[7] = lam * d[2] / T;
    x[8] = lam * d[3] / qs;
    x[9] = lam * d[4] / (n * T);
    x[10] = cc.denseness;
    x[11] = cc.log10kn;
    *scale = n * itau;
}

// Correction of the student's L[phi]: corr[i][k] (k < Q) = P (n / tau) (y * out_std +
// out_mean) on cells whose normalised inputs lie in [lo, hi]; zero (and counted in
// *outside) elsewhere.  The projection runs in FP64, so the mass, momentum and energy of
// the correction vanish to FP64 rounding before it is stored in the state's precision R.
// 64 cells per block.
template <typename R>
__global__ __launch_bounds__(256) void k_closure_apply(const unsigned short *wb, const float *params,
                                                       const float *norm, const double *Pc,
                                                       const double *rows5, ClosureConst cc, int nx,
                                                       int Q, R *corr,
                                                       unsigned long long *outside)
{
    __shared__ MlpSmem s;
    __shared__ float ys[4][16 * 17];
    __shared__ double sc[4][16];
    __shared__ int in_hull[4][16];
    __shared__ double pcs[MLP_OUT * MLP_OUT];
    mlp_stage_weights(s, wb, params);
    for (int j = threadIdx.x; j < MLP_OUT * MLP_OUT; j += blockDim.x) pcs[j] = Pc[j];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cell0 = blockIdx.x * MLP_ROWS + wave * 16;
    for (int j = lane; j < 16 * MLP_K1; j += 64) s.act[wave][0][(j / MLP_K1) * AS + j % MLP_K1] = 0;
    __syncthreads();
    if (lane < 16) {
        const int i = cell0 + lane;
        int inside = 0;
        double scale = 0.0;
        if (i < nx) {
            double x[MLP_IN], sd;
            closure_features(rows5, i, cc, x, &sd);
            inside = 1;
            for (int c = 0; c < MLP_IN; ++c) {
                float v = ((float)x[c] - norm[NRM_IN_MEAN + c]) / norm[NRM_IN_STD + c];
                if (!(v >= norm[NRM_LO + c] && v <= norm[NRM_HI + c])) inside = 0;
                s.act[wave][0][lane * AS + c] = f2bf(v);
            }
            scale = sd;
        }
        sc[wave][lane] = scale;
        in_hull[wave][lane] = inside;
    }
    __syncthreads();
    floatx4 o;
    mlp_forward_rows(s, wave, lane, nullptr, 0, 16, o);
    {
        const int col = lane & 15, rq = 4 * (lane >> 4);
#pragma unroll
        for (int r = 0; r < 4; ++r) ys[wave][(rq + r) * 17 + col] = o[r];
    }
    __syncthreads();
    if (lane < 16) {
        const int i = cell0 + lane;
        if (i < nx) {
            const bool inside = in_hull[wave][lane] != 0;
            double v[MLP_OUT];
            for (int o2 = 0; o2 < MLP_OUT; ++o2)
                v[o2] = o2 < Q ? sc[wave][lane] * (double)(ys[wave][lane * 17 + o2] * norm[NRM_OUT_STD + o2] +
                                                           norm[NRM_OUT_MEAN + o2])
                               : 0.0;
            for (int k = 0; k < Q; ++k) {
                double acc = 0.0;
                for (int o2 = 0; o2 < Q; ++o2) acc += pcs[k * MLP_OUT + o2] * v[o2];
                corr[(size_t)i * Q + k] = inside ? (R)acc : R(0);
            }
            if (!inside) atomicAdd(outside, 1ull);
        }
    }
}

// Training sample of every cell: x[i] = the 12 inputs, y[i][j] = (Lt[i][j] - Ls[i][j]) tau / n
// for j < Q (Lt: the projected teacher right-hand side, Ls: the student's; both rows of
// stride ls).
__global__ void k_closure_sample(const double *rows5, ClosureConst cc, int nx, int Q,
                                 const double *Lt, const double *Ls, int ls, float *x_out,
                                 float *y_out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx) return;
    double x[MLP_IN], sd;
    closure_features(rows5, i, cc, x, &sd);
    for (int c = 0; c < MLP_IN; ++c) x_out[(size_t)i * MLP_IN + c] = (float)x[c];
    for (int j = 0; j < Q; ++j)
        y_out[(size_t)i * Q + j] = (float)((Lt[(size_t)i * ls + j] - Ls[(size_t)i * ls + j]) / sd);
}

// out[r][j] = sum_k P[j][k] in[r][k] for rows r < nrows (FP64), j < qo, k < qi.
__global__ void k_project_rows(const double *P, const double *in, int in_stride, int qi, double *out,
                               int out_stride, int qo, int nrows)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (size_t)nrows * qo) return;
    const int r = (int)(t / qo), j = (int)(t - (size_t)r * qo);
    double s = 0.0;
    for (int k = 0; k < qi; ++k) s += P[(size_t)j * qi + k] * in[(size_t)r * in_stride + k];
    out[(size_t)r * out_stride + j] = s;
}

// d[r][c] = a[r][c] - b[r][c] over rows r < nrows of width w (FP64).
__global__ void k_diff_rows(const double *a, const double *b, double *d, int w, int nrows)
{
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (size_t)nrows * w) d[t] = a[t] - b[t];
}

}  // namespace elb
