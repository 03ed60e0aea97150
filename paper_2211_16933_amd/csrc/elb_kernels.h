// Device kernels of the FDLB step (gfx950).  Included by elb.hip only.
//
// Layout in HBM: a distribution level is (nx + 6) rows of 2Q values, row r = cell r - 3,
// each row [phi_0 .. phi_{Q-1}, theta_0 .. theta_{Q-1}] with the node index fastest.
// Rows 0..2 and nx+3..nx+5 are ghost cells (equilibrium boundaries; periodic problems
// wrap the cell index instead).  Three levels hold psi^n, psi^(1), psi^(2) of the RK3
// scheme; the last stage writes psi^{n+1} over psi^n in place (it reads psi^n only at its
// own cells).  The FP32 mode with conserved bookkeeping adds, per level, three FP64 values
// per row: n, n u and E = (n u^2 + 3 n T)/2.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mlp_device.h"

namespace elb {

constexpr int NG = 3;  // ghost cells per side (the +-3 stencils of WENO-5 and FD6)

// MODE_FP32_FIXUP: MODE_FP32_MIXED plus the moment fix-up of the FP32 rows (phase A2)
enum { MODE_FP64 = 0, MODE_FP32 = 1, MODE_FP32_MIXED = 2, MODE_FP32_FIXUP = 3 };

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename R>
struct StageArgs {
    const R *psi_s;       // stage input level (read with +-3 halos)
    const R *psi_n;       // level n (read at own cells for the RK combination)
    R *psi_out;           // output level (interior rows only)
    const double *U_s;    // bookkeeping mode: conserved (n, nu, E) per row, stage input
    const double *U_n;    // bookkeeping mode: level n
    double *U_out;        // bookkeeping mode: output level
    const double *p;      // nodes p_k
    const double *w;      // quadrature weights w_k (bookkeeping: moment fix-up)
    const R *Bt;          // Bt[l][k] = w_k He_l(p_k)/sqrt(l!) (zero outside l<=N, k<Q), packed
                          // per MFMA lane, split by parity when Q/2 % 16 == 0 (phase C)
    const double *cref;   // deviation storage: n_r c_l(u_r, T_r), l < Qp
    const double *gref;   // deviation storage: n_r g_k(u_r, T_r), k < Q
    const double *rec;    // [2][Qp]: 1/sqrt(l) and sqrt(l/(l+1)) (recurrence constants)
    int *flag;            // set to 1 when a cell has n <= 0, T <= 0 or non-finite moments
    int nx, N, periodic, pr_enskog;
    double dx, dt, b, mu_ref, pr;
    double a_n, a_s, a_L; // psi_out = a_n psi^n + a_s psi^(s) + a_L dt L[psi^(s)], a_n + a_s = 1
    double T_ref;         // deviation storage: reference temperature
    double ref_sum[6];    // deviation storage: S_0..S_3 and R_0, R_1 of psi_ref
    const R *corr;        // learned closure: [nx][Q] added to L[phi] (NULL: none)
    // learned closure evaluated inside the stage (fused form): the network's bfloat16
    // weights and FP32 parameters, its normalisation block, the projector Pc [16][16], the
    // inputs E_l and log10 Kn, and the count of cells outside the training range
    const unsigned short *mwb;
    const float *mparams, *mnorm;
    const double *mpc;
    double cl_denseness, cl_log10kn;
    unsigned long long *outside;
    const double *fm_w;   // chi_RET-FM: weights w_{-J..J} of the ball average (RET kernels only)
    int fm_J;             // and its half-width J
    // FP32 storage: the stochastic rounding stream of this launch is seed (+ *seed_base when
    // seed_base is not NULL: a captured graph keeps its offset in seed and reads the base)
    unsigned seed;
    const unsigned *seed_base;
};

constexpr int MAXQP = 208;

// Launch shape of the stage kernel for storage type R and Q nodes:
//   S strips of L cells per block (W = S L cells), 2Q columns (phi and theta of every node),
//   one thread per (column, strip) -> 2Q S threads.  W is a multiple of 16 (MFMA tiles).
template <typename R, int Q> struct Shape;
#define ELB_SHAPE(RT, QV, SV, LV) \
    template <> struct Shape<RT, QV> { static constexpr int S = SV, L = LV; };
// FP32: 8-cell strips in blocks of up to 768 threads (12 waves), two blocks per CU.  Q <= 20
// and Q = 32 on 8 strips (64-cell tiles), so that the 65536-cell tube has 1024 tiles rather
// than a single round of 512 (or 683 for Q = 32 on 12 strips), in which no later block hides
// the per-block phases
ELB_SHAPE(float, 8, 8, 8)
ELB_SHAPE(float, 12, 8, 8)
ELB_SHAPE(float, 16, 8, 8)
ELB_SHAPE(float, 20, 8, 8)
ELB_SHAPE(float, 24, 16, 8)
ELB_SHAPE(float, 32, 8, 8)
ELB_SHAPE(float, 40, 8, 8)
ELB_SHAPE(float, 48, 8, 8)
ELB_SHAPE(float, 64, 6, 8)
ELB_SHAPE(float, 96, 4, 8)
ELB_SHAPE(float, 200, 2, 8)
// FP64: the same strips, tiles bounded by LDS and, for Q <= 24, by the tile count of the
// 65536-cell tube (64 cells or fewer)
ELB_SHAPE(double, 8, 8, 8)
ELB_SHAPE(double, 12, 8, 8)
ELB_SHAPE(double, 16, 8, 8)
ELB_SHAPE(double, 20, 4, 8)
ELB_SHAPE(double, 24, 4, 8)
ELB_SHAPE(double, 32, 4, 8)
ELB_SHAPE(double, 40, 8, 8)
ELB_SHAPE(double, 48, 4, 8)
ELB_SHAPE(double, 64, 2, 8)
// Q = 96: 2 x 8 (6 waves, up to 96 registers, three blocks per CU); 4 x 8 held to 80
// registers spilled in the march
ELB_SHAPE(double, 96, 2, 8)
ELB_SHAPE(double, 200, 2, 8)
#undef ELB_SHAPE

template <typename R, int Q, int S_ = Shape<R, Q>::S, int L_ = Shape<R, Q>::L>
struct Geometry {
    static constexpr int S = S_, L = L_;
    static constexpr int W = S * L;             // cells per block
    static constexpr int C2 = 2 * Q;            // columns
    static constexpr int H = S * Q;             // (column, strip) items of one velocity sign
    // threads per block: each velocity sign's H items rounded up to whole waves (HW threads),
    // so that no wave holds items of both signs; the threads past H in each half own no
    // item and sit out the march (phases W, D)
    static constexpr int HW = (H + 63) / 64 * 64;
    static constexpr int NT = 2 * HW;
    // occupancy the register allocation is held to (waves per SIMD): two blocks of 10 or 12
    // waves (3 per SIMD each), three of 8 or three of 6 per CU; 1 = no constraint
    static constexpr int WV = (NT == 768 || NT == 640 || NT == 512) ? 6 : NT == 384 ? 5 : 1;
    // with the learned closure inside (Q <= 16): at least two blocks per CU, and four waves
    // per SIMD for blocks of up to four waves (four or more blocks per CU)
    static constexpr int WVCL0 = NT <= 256 ? 4 : (2 * NT / 64 + 3) / 4;
    static constexpr int WVCL = WVCL0 > WV ? WVCL0 : WV;
    // lanes per cell of the segmented coefficient recurrence: the largest of 8, 4, 2, 1 for
    // which the (cell, segment) items fit in the waves after those of the per-cell phase;
    // 16 when that still fits and takes at most four waves (16-cell tiles: shorter segments
    // for one more scan step; with more cells the extra waves cost more than they save)
    static constexpr int WC = (W + 63) / 64 * 64;
    static constexpr int RG = 16 * W <= 256 && 16 * W + WC <= NT ? 16
                            : 8 * W + WC <= NT ? 8 : 4 * W + WC <= NT ? 4 : 2 * W + WC <= NT ? 2 : 1;
    static constexpr int ROWS = W + 2 * NG;     // staged rows
    static constexpr int QP = (Q + 15) / 16 * 16;  // padded node count (MFMA tiles)
    // The nodes are symmetric (p_{Q-1-k} = -p_k, equal weights) and He_l has the parity of
    // l, so when Q/2 fills whole 16-wide MFMA tiles the projection splits into even and odd
    // orders over the QH = Q/2 positive nodes (half the work); then QP = 2 QH.
    static constexpr int QH = Q / 2;
    static constexpr bool SPLIT = QH % 16 == 0;
    // LDS row stride of the c buffer (coefficients; [even | odd] when split) and the g
    // buffer (g; [E | O] half sums when split): a multiple of 16 bytes (16-byte operand
    // reads), off a multiple of 32 banks
    static constexpr int GS = QP + 16 / (int)sizeof(R);
    // Every wave holds items of one velocity sign, so the upwind direction of the march is
    // uniform per wave (Q = 200: 400 items per sign in 7 waves each, the last one a quarter
    // full).
    static_assert(W % 16 == 0, "tile width must be a multiple of 16");
    static_assert(Q % 2 == 0, "even node counts only (no zero node)");
    static_assert(NT <= 1024, "block too large");
};

// --------------------------------------------------------------------------------------
// closures (Sec. II.A-B): chi_SET and 1/tau (the stage kernel forms them inline)
// --------------------------------------------------------------------------------------
__device__ inline double chi_set(double eta)
{
    double om = 1.0 - eta;
    return 0.5 * (2.0 - eta) / (om * om * om);
}

// 1/tau with tau = mu / (n T), mu = (mu_ref sqrt T / chi)(1 + 0.8 y + C y^2), y = b n chi
__device__ inline double inv_tau(double mu_ref, double n, double T, double chi, double y)
{
    const double cm = (4.0 / 25.0) * (1.0 + 12.0 / M_PI);
    return n * chi * sqrt(T) / (mu_ref * (1.0 + 0.8 * y + cm * y * y));
}

// reciprocal and ratio: IEEE division in FP64, the hardware reciprocal (1 ulp) in FP32
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double ratio(double a, double b) { return a / b; }
__device__ inline float ratio(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
// added to every scaled smoothness indicator: FP32 keeps indicators that vanish or underflow
// from producing infinite ratios; FP64 tests for exact zeros instead
template <typename R> struct IndFloor;
template <> struct IndFloor<float> { static constexpr float value = 1e-30f; };
template <> struct IndFloor<double> { static constexpr double value = 0.0; };

// Storage row of cell `cell` (may lie in the halo): periodic wrap or the ghost rows.
__device__ inline int row_of(int cell, int nx, int periodic)
{
    if (periodic) {
        int c = cell % nx;
        if (c < 0) c += nx;
        return c + NG;
    }
    return cell + NG;
}

__device__ inline floatx4 mfma16x16x4(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline doublex4 mfma16x16x4(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename R> struct Acc4;
template <> struct Acc4<float> { typedef floatx4 type; };
template <> struct Acc4<double> { typedef doublex4 type; };

// Lane exchanges on the DPP path of the vector ALU (no LDS traffic), inside rows of 16
// lanes.  gfx9 DPP controls: quad_perm [1,0,3,2] (partner lane ^ 1), quad_perm [2,3,0,1]
// (lane ^ 2), row_half_mirror (lane 7 - i within each 8), row_shr:n (lane i - n; lanes
// below n of a row keep the old value, here 0).
enum : int { DPP_X1 = 0xB1, DPP_X2 = 0x4E, DPP_MIR8 = 0x141, DPP_SHR = 0x110 };

template <int CTRL>
__device__ inline double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over a group of 8 aligned lanes, in every lane (partners 7 - i, i ^ 2, i ^ 1 span the
// group).
__device__ inline double sum8_dpp(double v)
{
    v += dpp_f64<DPP_MIR8>(v);
    v += dpp_f64<DPP_X2>(v);
    v += dpp_f64<DPP_X1>(v);
    return v;
}

// One doubling step of an inclusive scan of 2x2 matrices over groups of RG lanes (product
// with the matrix of lane g - D on the right); no-op when D >= RG.
template <int D, int RG>
__device__ inline void scan_step(double &x00, double &x01, double &x10, double &x11, int g)
{
    if constexpr (D < RG) {
        const double y00 = dpp_f64<DPP_SHR + D>(x00), y01 = dpp_f64<DPP_SHR + D>(x01);
        const double y10 = dpp_f64<DPP_SHR + D>(x10), y11 = dpp_f64<DPP_SHR + D>(x11);
        if (g >= D) {
            const double n00 = fma(x00, y00, x01 * y10), n01 = fma(x00, y01, x01 * y11);
            const double n10 = fma(x10, y00, x11 * y10), n11 = fma(x10, y01, x11 * y11);
            x00 = n00; x01 = n01; x10 = n10; x11 = n11;
        }
    }
}

// One halving exchange of a multi-value reduction over a lane group: lanes with `hi` set
// keep the upper half of their CNT values and send the lower half to the partner lane
// (DPP control CTRL, whose `hi` is the opposite), which does the opposite; each lane then
// holds CNT/2 partial sums over the pair.
template <int CNT, int CTRL>
__device__ inline void halve(double *v, bool hi)
{
#pragma unroll
    for (int q = 0; q < CNT / 2; ++q) {
        const double send = hi ? v[q] : v[q + CNT / 2];
        const double keep = hi ? v[q + CNT / 2] : v[q];
        v[q] = keep + dpp_f64<CTRL>(send);
    }
}

// Learned closure of the cells of a stage tile, the fused form of k_closure_apply: the
// normalised inputs cin [W][16] (12 inputs, then zeros) go through the network in 16-cell
// tiles, one per wave and pass, on v_mfma_f32_16x16x32_bf16 (weights read as bfloat16 from
// global memory, FP32 accumulation, bias and SiLU in FP32, activations rounded to
// bfloat16 in the wave's LDS tile act [16][AS], in place).  Then per cell, 4 lanes each,
// c[k] = sum_o Pc[k][o] (n / tau) (y_o sigma_o + mu_o), k < Q, in FP64, stored to
// corr [W][Q] (zero, and counted, for cells outside the training range).  The arithmetic
// and its order are those of k_closure_apply.  cst holds the Q rows of Pc [16][16] that are
// read (FP64), then as FP32 the normalisation block and the biases b1, b2, b3, b4, staged in
// LDS by phase 0.
// Operand lane layout: lane l holds A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16],
// i < 8; the result D[4 (l / 16) + r][l % 16] is acc[r].
constexpr int CL_PC = MLP_OUT * MLP_OUT;          // doubles of Pc [16][16]
constexpr int CL_NB = MLP_NORM + 3 * MLP_H + MLP_OUT;  // floats after them: norm, biases

template <typename R, int Q, int W, int NWAVE>
__device__ inline void closure_tile(const StageArgs<R> &a, const unsigned short *cin,
                                    const double *csc, const int *cok, const double *cst, R *corr,
                                    unsigned short *actbase, int wcount, int wave, int lane)
{
    const double *pc = cst;
    const float *nrm = reinterpret_cast<const float *>(cst + Q * MLP_OUT);
    const float *bias = nrm + MLP_NORM;  // b1, b2, b3 (64 each), b4 (16)
    unsigned short *act = actbase + wave * 16 * AS;
    float *ys = reinterpret_cast<float *>(act);  // the outputs [16][17], after the last layer
    const int col = lane & 15, rq = 4 * (lane >> 4), kq = 8 * (lane >> 4);
    // the weights of one layer (B operands) from global memory, 8 bfloat16 per lane and
    // 16-column block; `z` is an opaque zero ordered after a layer's input, so that the next
    // layer's weights load while this layer computes and not all of them ahead of the loop
    auto wld = [&](int off) {
        return __builtin_bit_cast(bf16x8, *reinterpret_cast<const ushort8 *>(a.mwb + off));
    };
    auto after = [](bf16x8 dep) {
        int z = 0;
        const float d = __builtin_bit_cast(floatx4, dep).x;
        asm volatile("" : "+v"(z) : "v"(d));
        return z;
    };
    const bf16x8 zero8 = __builtin_bit_cast(bf16x8, ushort8{0, 0, 0, 0, 0, 0, 0, 0});
    for (int t = wave; t < W / 16; t += NWAVE) {
        floatx4 acc[4];
        bf16x8 wa[8], wb[8];  // this layer's and the next layer's weights
        // layer 1 (K = 32; inputs 16..31 are zero and not stored)
        const bf16x8 a1 = kq < 16 ? ld8(cin + (t * 16 + col) * 16 + kq) : zero8;
        int z = after(a1);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) wa[tt] = wld(z + OFF_W1 + (tt * 16 + col) * MLP_K1 + kq);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
                wb[4 * kk + tt] = wld(z + OFF_W2 + (tt * 16 + col) * MLP_H + kk * 32 + kq);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
            acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, wa[tt], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int c = tt * 16 + col;
                act[(rq + r) * AS + c] = f2bf(silu(acc[tt][r] + bias[c]));
            }
        // layers 2 and 3 (K = 64), each read in full before the tile is overwritten (the
        // wave's LDS accesses execute in order)
#pragma unroll
        for (int l = 0; l < 2; ++l) {
            const bf16x8 av0 = ld8(act + col * AS + kq), av1 = ld8(act + col * AS + 32 + kq);
            z = after(av0);
#pragma unroll
            for (int u = 0; u < 8; ++u) wa[u] = wb[u];
            if (l == 0) {
#pragma unroll
                for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                    for (int tt = 0; tt < 4; ++tt)
                        wb[4 * kk + tt] = wld(z + OFF_W3 + (tt * 16 + col) * MLP_H + kk * 32 + kq);
            } else {
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) wb[kk] = wld(z + OFF_W4 + col * MLP_H + kk * 32 + kq);
            }
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av0, wa[tt], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                acc[tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av1, wa[4 + tt], acc[tt], 0, 0, 0);
            }
#pragma unroll
            for (int tt = 0; tt < 4; ++tt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int c = tt * 16 + col;
                    act[(rq + r) * AS + c] = f2bf(silu(acc[tt][r] + bias[(l + 1) * MLP_H + c]));
                }
        }
        // layer 4: 16 outputs
        floatx4 o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(act + col * AS + kq), wb[0],
                                                            floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(act + col * AS + 32 + kq), wb[1], o, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) ys[(rq + r) * 17 + col] = o[r] + bias[3 * MLP_H + col];
        // projection onto the moment-free subspace, 4 lanes per cell
        const int cell = lane >> 2, part = lane & 3, i = t * 16 + cell;
        if (i < wcount) {
            const bool inside = cok[i] != 0;
            const double sc = csc[i];
            double sum[(Q + 3) / 4];
#pragma unroll
            for (int j4 = 0; j4 < (Q + 3) / 4; ++j4) sum[j4] = 0.0;
#pragma unroll 4
            for (int o2 = 0; o2 < Q; ++o2) {
                const double v = sc * (double)(ys[cell * 17 + o2] * nrm[NRM_OUT_STD + o2] + nrm[NRM_OUT_MEAN + o2]);
#pragma unroll
                for (int j4 = 0; j4 < (Q + 3) / 4; ++j4) {
                    const int kc = part + 4 * j4;
                    if (kc < Q) sum[j4] += pc[kc * MLP_OUT + o2] * v;
                }
            }
#pragma unroll
            for (int j4 = 0; j4 < (Q + 3) / 4; ++j4) {
                const int kc = part + 4 * j4;
                if (kc < Q) corr[i * Q + kc] = inside ? (R)sum[j4] : R(0);
            }
            if (part == 0 && !inside) atomicAdd(a.outside, 1ull);
        }
    }
}

// --------------------------------------------------------------------------------------
// Incremental WENO-5 (App. A.2) along a march.  For the upwind-ordered stencil
// (v0, v1, v2, v3, v4) of an interface, with second differences a1 = v0 - 2v1 + v2,
// a2 = v1 - 2v2 + v3, a3 = v2 - 2v3 + v4 and first differences d_jk = v_k - v_j, the
// smoothness indicators (App. A.2, times 12) are 13 a_q^2 + 3 c_q^2 with
// c1 = v0 - 4v1 + 3v2 = a1 + 2 d12, c2 = v1 - v3 = -(d12 + d23), c3 = 3v2 - 4v3 + v4 =
// a3 - 2 d23, and the candidate stencils are 6 v2 + h_q with h1 = 2v0 - 7v1 + 5v2 =
// 2 a1 + 3 d12, h2 = -v1 - v2 + 2v3 = d12 + 2 d23, h3 = -4v2 + 5v3 - v4 = 4 d23 - d34.
// The indicators are used divided by 36 (times 1/3), e_q + c_q^2 with e_q = (13/3) a_q^2:
// the weights depend on their ratios only.  The next interface along the march has the
// stencil (v1, v2, v3, v4, v5), so a2, a3, e2, e3 and d23, d34 carry over and one new value
// enters per step.
//
// Weights (eq. weno5_omega): (delta_q / varphi_q^2) / sum, evaluated as delta_q r_q^2 / sum
// with r_q = min_s varphi_s / varphi_q.  FP64: r_q = 1 where varphi_q == 0, which gives the
// Table III limits exactly.  FP32: each e_q carries 1e-30, which leaves every weight
// unchanged to FP32 precision when the indicators are representable and yields the Table
// III limits when some of them underflow.
// --------------------------------------------------------------------------------------
// two floats in the bytes of one double (float x at the lower address)
__device__ inline double pack_f2(float x, float y)
{
    return __hiloint2double(__float_as_int(y), __float_as_int(x));
}

// 32-bit integer mix (xor-shift / multiply rounds of the "lowbias32" finaliser, C. Wellons):
// a counter-based source of pseudo-random words for the stochastic rounding of FP32 stores
__device__ inline unsigned mix32(unsigned x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <typename R>
struct WenoMarch {
    R v2, v3, v4;     // last three values of the current stencil
    R a2, a3;         // second differences (v1,v2,v3), (v2,v3,v4)
    R e2, e3;         // (13/3) a2^2, (13/3) a3^2 (plus the FP32 floor)
    R d23, d34;       // first differences v3 - v2, v4 - v3
    R d12;            // v2 - v1

    // zero state; five shift() calls then hold the stencil of the five values shifted in
    __device__ inline void zero()
    {
        v2 = v3 = v4 = R(0);
        a1_ = a2 = a3 = R(0);
        e1_ = e2 = e3 = R(0);
        d12 = d23 = d34 = R(0);
    }
    // 6 x the interpolant at the interface of the current stencil
    __device__ inline R interp6() const
    {
        const R c1 = fma(R(2), d12, a1_);
        const R c2 = d12 + d23;
        const R c3 = fma(R(-2), d23, a3);
        const R s1 = fma(c1, c1, e1_);
        const R s2 = fma(c2, c2, e2);
        const R s3 = fma(c3, c3, e3);
        R t1, t2, t3;
        weights(s1, s2, s3, t1, t2, t3);
        R h1 = R(2) * a1_ + R(3) * d12;
        R h2 = d12 + R(2) * d23;
        R h3 = R(4) * d23 - d34;
        R num = t1 * h1 + t2 * h2 + t3 * h3;
        return R(6) * v2 + num * recip(t1 + t2 + t3);
    }
    // advance to the next interface with the entering value v5
    __device__ inline void shift(R v5)
    {
        const R d45 = v5 - v4;
        const R a4 = d45 - d34;
        a1_ = a2; e1_ = e2;
        a2 = a3; e2 = e3;
        a3 = a4; e3 = fma(R(13.0 / 3.0) * a4, a4, IndFloor<R>::value);
        d12 = d23; d23 = d34; d34 = d45;
        v2 = v3; v3 = v4; v4 = v5;
    }
    R a1_, e1_;

    static __device__ inline void weights(R s1, R s2, R s3, R &t1, R &t2, R &t3)
    {
        if constexpr (sizeof(R) == 4) {
            R mn = fmin(s1, fmin(s2, s3));
            R r1 = mn * recip(s1), r2 = mn * recip(s2), r3 = mn * recip(s3);
            t1 = R(0.1) * r1 * r1; t2 = R(0.6) * r2 * r2; t3 = R(0.3) * r3 * r3;
        } else {
            // FP64 with one division: with g_q = varphi_q / min varphi >= 1, the weights
            // delta_q / g_q^2 are proportional to delta_q prod_{p != q} g_p^2.  g is clamped at
            // 1e50: a weight 1e-100 below the largest is zero at FP64 precision, and the
            // products stay below 1e200.  If some indicator vanishes, the weights are
            // delta_q on the zero set and 0 elsewhere (Table III limits).
            const R mn = fmin(s1, fmin(s2, s3));
            const bool z = mn == R(0);
            const R im = R(1) / (z ? R(1) : mn);
            const R g1 = fmin(s1 * im, R(1e50)), g2 = fmin(s2 * im, R(1e50)), g3 = fmin(s3 * im, R(1e50));
            const R q1 = g1 * g1, q2 = g2 * g2, q3 = g3 * g3;
            t1 = z ? (s1 == R(0) ? R(0.1) : R(0)) : R(0.1) * (q2 * q3);
            t2 = z ? (s2 == R(0) ? R(0.6) : R(0)) : R(0.6) * (q1 * q3);
            t3 = z ? (s3 == R(0) ? R(0.3) : R(0)) : R(0.3) * (q1 * q2);
        }
    }
};

// --------------------------------------------------------------------------------------
// One RK3 stage for a tile of W cells (one block).
//
// FP32 storage holds deviations from a fixed reference equilibrium psi_ref (one constant
// per column; phi_ref_k = n_r g_k(u_r, T_r), theta_ref_k = 2 T_r phi_ref_k), so that small
// departures from the reference keep FP32 relative precision.  WENO-5 acts on the
// deviation unchanged (its smoothness indicators use differences only, and the candidate
// stencils reproduce constants), moments add the FP64 reference sums, and the equilibrium is
// formed as a deviation through the coefficient difference n c_l(u,T) - n_r c_l(u_r,T_r).
// FP64 storage holds psi itself (reference zero).
//
// Thread roles in the march: the first half of the block takes the columns of the nodes
// with p_k < 0 (phi and theta), the second half p_k > 0, each as (column, strip) items, so
// the upwind direction is uniform in every wave; negative-velocity items march right to
// left, positive ones left to right, always upwind-first.
//
//   phase 0  stage rows [i0-3, i0+W+3) of psi^(s) in LDS (16-byte loads)
//   phase A  per row: FP64 sums S_j = sum p^j phi (j <= 3), R_j = sum p^j theta (j <= 1);
//            8 (or 4) lanes per row over node pairs (k, Q-1-k), one pass over all rows
//   phase W  each item copies its column window (L + 6 values) from LDS to registers
//   phase A2 per row: n, u, T, q (Sec. II.D); with bookkeeping n, u, T come from the FP64
//            conserved densities of the row and q from the sums
//   phase B  per cell: closures, FD6 gradients of ln n, u, ln T (App. A.3) (CL: then the
//            learned closure's inputs, in a pass of their own), and the
//            Hermite coefficients c_l = sqrt(l!) a_l(u, T) in FP64, where a_l is the inner
//            sum of eq. g_alpha; a_l is the Taylor coefficient of exp(u t + (T-1) t^2/2),
//            whose derivative gives (l+1) a_{l+1} = u a_l + (T-1) a_{l-1}
//   phase C  g = c Bt on the matrix cores: [W x Qp] x [Qp x Qp], 16x16x4 MFMA tiles
//   phase L  (CL) the learned closure: the network on the inputs phase B formed, then the
//            projected correction of L[phi] per cell (closure_tile)
//   phase D  per item: march along the strip with the register window, one WENO-5
//            interpolant per interface, Shakhov target, J1 and the RK combination
//   phase E  (bookkeeping) per interface FP64 sums of the flux moments, then per cell
//            U_out = a_n U^n + a_s U^(s) + a_L dt (-(G_{i+1/2} - G_{i-1/2})/dx + J1 moments)
// --------------------------------------------------------------------------------------
template <typename R, int Q, int S_, int L_, int MODE, bool RET = false, bool CL = false>
__device__ __forceinline__ void stage_tile(const StageArgs<R> &a, const int blk)
{
    using G = Geometry<R, Q, S_, L_>;
    constexpr int W = G::W, C2 = G::C2, NT = G::NT, ROWS = G::ROWS, QP = G::QP, GS = G::GS;
    constexpr int QH = G::QH;
    constexpr bool SPLIT = G::SPLIT;
    constexpr int RG = G::RG;
    constexpr int S = G::S, L = G::L, H = G::H;
    constexpr bool BOOK = MODE == MODE_FP32_MIXED || MODE == MODE_FP32_FIXUP;
    constexpr bool FIX = MODE == MODE_FP32_FIXUP;
    constexpr bool DEV = sizeof(R) == 4;                     // deviation storage
    constexpr int NWAVE = NT / 64;
    constexpr bool PADDED = NT != 2 * H;                     // threads without an item
    // LDS row stride of the staged tile: padded by 32 bytes so that the 8 lanes of one row in
    // the moment pass and the 4 rows of a half-wave fall on distinct banks
    constexpr int TS = C2 + 32 / (int)sizeof(R);
    // LDS row stride of the bookkeeping's flux rows: when 2Q is a multiple of the 64 banks,
    // padded by 8 values, so that the 8 interfaces of a wave in phase E (8 lanes each) fall
    // on distinct banks
    constexpr int FS = C2 % 64 == 0 ? C2 + 8 : C2;
    constexpr int FB = BOOK ? (W + 1) * FS : 0;              // flux values (bookkeeping)
    // CL: the fused learned closure, whose activation tiles (one per wave) take the
    // coefficient buffer once the projection has read it
    static_assert(!CL || Q <= MLP_OUT, "the learned closure takes Q <= 16");
    constexpr int CLA = CL ? (NWAVE * 16 * AS * 2 + (int)sizeof(R) - 1) / (int)sizeof(R) : 0;
    constexpr int CB0 = W * GS > FB ? W * GS : FB;
    constexpr int CB = CB0 > CLA ? CB0 : CLA;                // coefficients, later fluxes
    constexpr int AREA = ROWS * TS > CB + W * GS ? ROWS * TS : CB + W * GS;
    constexpr int RL = Q % 8 == 0 ? 8 : 4;  // lanes per row of the moment pass
    static_assert(Q % RL == 0, "phi and theta columns split evenly over the row lanes");

    // The tile (phases 0-W) and, once every item holds its window in registers, the
    // coefficient/flux buffer and the equilibrium buffer (phases B-E) share one area.
    __shared__ __attribute__((aligned(16))) R area[AREA];
    R *const tile = area;
    R *const cbuf = area;
    R *const gbuf = area + CB;
    __shared__ double pk_s[Q];
    __shared__ double rec_s[2 * QP];  // 1/sqrt(l) and sqrt(l/(l+1)), l < QP
    __shared__ double cref_s[DEV ? QP : 1];
    __shared__ double gref_s[DEV ? Q : 1];   // n_r g_k(u_r, T_r), read by the march
    __shared__ __attribute__((aligned(16))) double red[ROWS * 6];
    __shared__ double r_n[ROWS], r_u[ROWS], r_T[ROWS], r_q[ROWS], r_lnn[ROWS], r_lnT[ROWS];
    __shared__ __attribute__((aligned(16))) R cellv[W * 16];
    __shared__ double jm[BOOK ? 2 * W : 1];
    __shared__ double gsum[BOOK ? 3 * (W + 1) : 1];
    __shared__ double ucell[BOOK ? 6 * W : 1];  // bookkeeping: U^(s), then U^n of the cells
    // the weights w_k of the moment fix-up (phase A2)
    __shared__ double w_s[FIX ? Q : 1];
    // CL: Pxx of the staged rows, the normalised bfloat16 inputs of every cell (12, then
    // zeros), its n / tau and inside flag, and the correction of L[phi] [W][Q]
    __shared__ double r_pxx[CL ? ROWS : 1];
    __shared__ __attribute__((aligned(16))) unsigned short cin_s[CL ? W * 16 : 8];
    __shared__ double csc_s[CL ? W : 1];
    __shared__ int cok_s[CL ? W : 1];
    __shared__ R corr_s[CL ? W * Q : 1];
    // CL: the closure's constants (Pc, then as FP32 the normalisation block and the biases)
    constexpr int CLP = Q * MLP_OUT;  // doubles of the Pc rows k < Q (the ones read)
    __shared__ double cst_s[CL ? CLP + (CL_NB + 1) / 2 : 1];
    // phase 0 sends the stores of threads with nothing to store to a 64-slot sink in red,
    // which is filled only in phase A
    static_assert(sizeof(double) * ROWS * 6 >= 64 * 16, "the sink fits in red");
    floatx4 *const sink = reinterpret_cast<floatx4 *>(red);

    // Wave priority: the phases before and after the march run chains of dependent
    // instructions on one or a few waves, while the march of another block on the same CU
    // keeps its waves always ready; those phases run at a raised priority, so that their
    // chains issue first and the march fills the remaining issue slots.
    __builtin_amdgcn_s_setprio(2);
    const int nx = a.nx;
    const int i0 = blk * W;
    // stochastic rounding stream of this launch (FP32 storage)
    const unsigned sd = DEV ? a.seed + (a.seed_base ? *a.seed_base : 0u) : 0u;
    const int wcount = min(W, nx - i0);
    const int rows = wcount + 2 * NG;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    // item of this thread: sign half, distribution (phi or theta), strip and node.  When the
    // S Q/2 items of one sign and one distribution fill whole waves (THW), each wave holds
    // items of one distribution only, and the march is compiled for it; otherwise the
    // distribution is chosen per lane.
    constexpr int HQ = S * (Q / 2);
    constexpr bool THW = HQ % 64 == 0;
    const bool neg = tid < G::HW;
    const int it = neg ? tid : tid - G::HW;   // it >= H (ds >= S): no item
    int ds, jn;
    bool isth;
    if constexpr (THW) {
        isth = it >= HQ;
        const int r = isth ? it - HQ : it;
        ds = r / (Q / 2);
        jn = r - ds * (Q / 2);
    } else {
        ds = it / Q;
        const int jq = it - ds * Q;
        isth = jq >= Q / 2;
        jn = isth ? jq - Q / 2 : jq;
    }
    const int k = (neg ? 0 : Q / 2) + jn;
    const int dc = (isth ? Q : 0) + k;
    const int ib = ds * L;
    // the same sign and distribution as scalars of the wave (the branches on them are uniform)
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    const bool neg_w = wv < G::HW / 64;
    const bool th_w = THW && (wv - (neg_w ? 0 : G::HW / 64)) * 64 >= HQ;

    // ---- phase 0: every global load of the phase (tile and node tables) is issued before
    // the first LDS store, so the block waits for memory once.  A thread past the end of a
    // table or of the staged rows loads a clamped (valid) entry and stores it into `sink`
    // (slot = its lane): the stores need no branch, so the loads stay ahead of them.
    static_assert(2 * QP <= NT, "one table entry per thread");
    {
        constexpr int VPR = C2 * sizeof(R) / 16;  // 16-byte vectors per row
        constexpr int VTS = TS * sizeof(R) / 16;
        constexpr int NLD = (ROWS * VPR + NT - 1) / NT;  // tile vectors per thread
        // clang vector types (not float4 structs), so the register array below stays in
        // registers
        const floatx4 *src = reinterpret_cast<const floatx4 *>(a.psi_s);
        floatx4 *dst = reinterpret_cast<floatx4 *>(tile);
        floatx4 *const sinkv = sink + lane;
        const int nv = rows * VPR;
        // source offsets first, then the loads back to back.  Unless a periodic tile wraps
        // round the domain, the staged rows are the storage rows i0 .. i0 + rows - 1 in order.
        const bool contiguous = !a.periodic || (i0 >= NG && i0 + wcount + NG <= nx);
        size_t off[NLD];
        if (contiguous) {
#pragma unroll
            for (int u = 0; u < NLD; ++u) off[u] = (size_t)i0 * VPR + min(tid + u * NT, nv - 1);
        } else {
#pragma unroll
            for (int u = 0; u < NLD; ++u) {
                const int idx = min(tid + u * NT, nv - 1);
                const int j = idx / VPR, v = idx - j * VPR;
                off[u] = (size_t)row_of(i0 - NG + j, nx, a.periodic) * VPR + v;
            }
        }
        floatx4 buf[NLD];
#pragma unroll
        for (int u = 0; u < NLD; ++u) buf[u] = src[off[u]];
        const double pkv = a.p[min(tid, Q - 1)];
        const double recv = a.rec[min(tid, 2 * QP - 1)];
        const double crefv = DEV ? a.cref[min(tid, QP - 1)] : 0.0;
        const double grefv = DEV ? a.gref[min(tid, Q - 1)] : 0.0;
        const double wv = FIX ? a.w[min(tid, Q - 1)] : 0.0;
        double *const sinkd = reinterpret_cast<double *>(sink) + lane;
        // when the block is a whole number of rows wide, every load of a thread falls in the
        // same column of the tile, NT / VPR rows apart
        constexpr bool EVEN = NT % VPR == 0;
        const int j0 = tid / VPR, v0 = tid - j0 * VPR;
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            const int idx = tid + u * NT;
            int j, v;
            if constexpr (EVEN) {
                j = j0 + u * (NT / VPR);
                v = v0;
            } else {
                j = idx / VPR;
                v = idx - j * VPR;
            }
            *(idx < nv ? dst + (j * VTS + v) : sinkv) = buf[u];
        }
        *(tid < Q ? pk_s + tid : sinkd) = pkv;
        *(tid < 2 * QP ? rec_s + tid : sinkd) = recv;
        if constexpr (DEV) {
            *(tid < QP ? cref_s + tid : sinkd) = crefv;
            *(tid < Q ? gref_s + tid : sinkd) = grefv;
        }
        if constexpr (FIX) *(tid < Q ? w_s + tid : sinkd) = wv;
        if constexpr (CL) {
            float *nb = reinterpret_cast<float *>(cst_s + CLP);
            for (int x = tid; x < CLP + CL_NB; x += NT) {
                if (x < CLP) {
                    cst_s[x] = a.mpc[x];
                } else {
                    const int y = x - CLP;
                    nb[y] = y < MLP_NORM ? a.mnorm[y]
                          : y < MLP_NORM + MLP_H ? a.mparams[OFF_B1 + y - MLP_NORM]
                          : y < MLP_NORM + 2 * MLP_H ? a.mparams[OFF_B2 + y - MLP_NORM - MLP_H]
                          : y < MLP_NORM + 3 * MLP_H ? a.mparams[OFF_B3 + y - MLP_NORM - 2 * MLP_H]
                          : a.mparams[OFF_B4 + y - MLP_NORM - 3 * MLP_H];
                }
            }
        }
    }
    __syncthreads();

    // bookkeeping: the tracked (n, nu, E) of staged row `tid` (phase A2), loaded now so that
    // the load overlaps phase A
    static_assert(ROWS <= NT, "one staged row per thread in phase A2");
    double Upre[3] = {0.0, 0.0, 0.0};
    if constexpr (BOOK) {
        if (tid < rows) {
            const double *Up = a.U_s + 3 * (size_t)row_of(i0 - NG + tid, nx, a.periodic);
            Upre[0] = Up[0];
            Upre[1] = Up[1];
            Upre[2] = Up[2];
        }
    }

    // ---- phase A: RL lanes per row; lane m sums columns m, m+RL, ... of the phi half and of
    // the theta half (Q % RL == 0, so a lane's phi and theta columns are the same nodes);
    // the partial sums are reduced over the RL lanes by halving exchanges
    for (int base = 0; base < rows * RL; base += NT) {
        const int t = base + tid;
        const int j = t / RL, m = t % RL;
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (j < rows) {
            const R *row = tile + j * TS;
            if constexpr ((Q / 2) % RL == 0) {
                // node pairs (k, Q - 1 - k), p_{Q-1-k} = -p_k: the even powers take the sum of
                // the pair, the odd powers the difference
#pragma unroll
                for (int x = 0; x < Q / (2 * RL); ++x) {
                    const int kk = m + RL * x;
                    const double pk = pk_s[kk], pp = pk * pk;
                    const double fa = (double)row[kk], fb = (double)row[Q - 1 - kk];
                    const double ta = (double)row[Q + kk], tb = (double)row[2 * Q - 1 - kk];
                    const double fs = fa + fb, pd = pk * (fa - fb);
                    v[0] += fs;
                    v[1] += pd;
                    v[2] = fma(pp, fs, v[2]);
                    v[3] = fma(pp, pd, v[3]);
                    v[4] += ta + tb;
                    v[5] = fma(pk, ta - tb, v[5]);
                }
            } else {
#pragma unroll
                for (int x = 0; x < Q / RL; ++x) {
                    const int kk = m + RL * x;
                    const double pk = pk_s[kk];
                    const double f = (double)row[kk];
                    const double ft = (double)row[Q + kk];
                    const double pf = pk * f;
                    v[0] += f;
                    v[1] += pf;
                    v[2] = fma(pk, pf, v[2]);
                    v[3] = fma(pk * pk, pf, v[3]);
                    v[4] += ft;
                    v[5] = fma(pk, ft, v[5]);
                }
            }
        }
        if constexpr (RL == 8) {
            // partners 7 - m, m ^ 2, m ^ 1: the three exchanges cover the 8 lanes of the row
            halve<8, DPP_MIR8>(v, m & 4);
            halve<4, DPP_X2>(v, m & 2);
            halve<2, DPP_X1>(v, m & 1);
            // lane 8r + m holds value 4 (m>>2 & 1) + 2 (m>>1 & 1) + (m & 1) = m
            if (j < rows && m < 6) red[j * 6 + m] = v[0];
        } else {
            halve<8, DPP_X2>(v, m & 2);
            halve<4, DPP_X1>(v, m & 1);
            // lane 4r + m holds values 2m and 2m + 1
            if (j < rows && 2 * m < 6) {
                red[j * 6 + 2 * m] = v[0];
                red[j * 6 + 2 * m + 1] = v[1];
            }
        }
    }

    // ---- phase W: the column window f_{ib-3} .. f_{ib+L+2} of this item.  In a partial
    // tile, rows past the staged ones hold stale values of the tile area: they enter only
    // interfaces and cells beyond the tile, which are never stored or summed.
    R win[L + 6];
#pragma unroll
    for (int x = 0; x < L + 6; ++x) {
        if constexpr (PADDED) win[x] = (ds < S && ib + x < rows) ? tile[(ib + x) * TS + dc] : R(0);
        else win[x] = tile[(ib + x) * TS + dc];
    }
    __syncthreads();  // tile area free from here on

    // ---- phase A2 (rows) and zero padding of the coefficient buffer, needed only when the
    // expansion stops short of the padded node count (rows of cells beyond a partial tile
    // give equilibria of cells that are never stored)
    if (a.N + 1 < QP)
        for (int idx = tid; idx < W * GS; idx += NT) cbuf[idx] = R(0);
    for (int j = tid; j < rows; j += NT) {
        double S0 = red[j * 6 + 0], S1 = red[j * 6 + 1], S2 = red[j * 6 + 2];
        double S3 = red[j * 6 + 3], R0 = red[j * 6 + 4], R1 = red[j * 6 + 5];
        if constexpr (DEV) {
            S0 += a.ref_sum[0]; S1 += a.ref_sum[1]; S2 += a.ref_sum[2];
            S3 += a.ref_sum[3]; R0 += a.ref_sum[4]; R1 += a.ref_sum[5];
        }
        double n, u, T;
        if constexpr (BOOK) {
            const double *U = Upre;  // row j = tid
            n = U[0];
            const double in = 1.0 / n;
            u = U[1] * in;
            T = (2.0 * U[2] * in - u * u) * (1.0 / 3.0);
            if constexpr (FIX) {
                // Moment fix-up: the FP32 row drifts from the tracked (n, nu, E) by
                // rounding.  phi_k += w_k (alpha + beta p_k) and theta_k += w_k eps restore
                // them exactly on the quadrature (sum w = 1, sum w p = 0, sum w p^2 = 1,
                // sum w p^3 = 0): alpha fixes n, beta fixes nu, and eps = 2 dE - alpha the
                // energy; the sums below become those of the fixed row.  Applied to the
                // stencil windows after this phase.
                const double al = U[0] - S0, be = U[1] - S1;
                const double ep = 2.0 * U[2] - (S2 + R0) - al;
                S0 += al;
                S1 += be;
                S2 += al;
                S3 += 3.0 * be;
                R0 += ep;
                // as four floats in the last 16 bytes of this row's slot of red (read above
                // by this thread only; 16-byte aligned, the slots are 48 bytes), written
                // through the slot's own type
                red[6 * j + 4] = pack_f2((float)al, (float)be);
                red[6 * j + 5] = pack_f2((float)ep, 0.0f);
            }
            if (j >= NG && j < NG + wcount) {
                ucell[3 * (j - NG) + 0] = U[0];
                ucell[3 * (j - NG) + 1] = U[1];
                ucell[3 * (j - NG) + 2] = U[2];
            }
        } else {
            n = S0;
            const double in = 1.0 / n;
            u = S1 * in;
            T = (S2 - n * u * u + R0) * in * (1.0 / 3.0);  // (3/2) n T = sum (xi^2 phi + theta)/2
        }
        double q = 0.5 * (S3 - 3.0 * u * S2 + 3.0 * u * u * S1 - u * u * u * S0) +
                   0.5 * (R1 - u * R0);         // sum xi (xi^2 phi + theta)/2
        double pxx = CL ? S2 - 2.0 * u * S1 + u * u * S0 : 0.0;  // sum xi^2 phi
        if (!(n > 0.0) || !(T > 0.0) || !isfinite(q) || !isfinite(u)) {
            atomicOr(a.flag, 1);
            n = 1.0; T = 1.0; u = 0.0; q = 0.0; pxx = 1.0;  // keep the block finite
        }
        if constexpr (CL) r_pxx[j] = pxx;
        r_n[j] = n;
        r_u[j] = u;
        r_T[j] = T;
        r_q[j] = q;
        r_lnn[j] = log(n);
        r_lnT[j] = log(T);
    }
    __syncthreads();

    // the moment fix-up of every staged row, applied to this item's window (phi:
    // w_k (alpha + beta p_k); theta: w_k eps), so that the march and the cell update see
    // rows whose n, nu and E are the tracked ones
    if constexpr (FIX) {
        if (!PADDED || ds < S) {
            const float wk = (float)w_s[k];
            const float wp = isth ? 0.0f : wk * (float)pk_s[k];
            const float wa = isth ? 0.0f : wk;
            const float we = isth ? wk : 0.0f;
#pragma unroll
            for (int x = 0; x < L + 6; ++x) {
                if (ib + x < rows) {
                    const floatx4 f = *reinterpret_cast<const floatx4 *>(red + 6 * (ib + x) + 4);
                    win[x] += wa * f.x + wp * f.y + we * f.z;
                }
            }
        }
    }

    // ---- phase R (chi_RET-FM only): the density of the J cells beyond each side of the
    // staged rows (one wave per cell, FP64 sums; with bookkeeping the tracked n), then per
    // staged row nbar = sum_{|m|<=J} w_m n_{c+m}, chi = chi_SET(b nbar / 4) and ln chi.
    // Dynamic LDS: w[2J+1], n over the cells i0-3-J .. i0+wcount+2+J, chi[ROWS], ln chi[ROWS].
    double *rchi = nullptr, *rlnchi = nullptr;
    if constexpr (RET) {
        extern __shared__ double fm_s[];
        const int J = a.fm_J;
        double *wts = fm_s;
        double *next = wts + (2 * J + 1);
        rchi = next + (2 * J + ROWS);
        rlnchi = rchi + ROWS;
        for (int idx = tid; idx <= 2 * J; idx += NT) wts[idx] = a.fm_w[idx];
        for (int j = tid; j < rows; j += NT) next[J + j] = r_n[j];
        for (int e = wave; e < 2 * J; e += NWAVE) {
            const bool left = e < J;
            const int c = left ? i0 - NG - J + e : i0 + wcount + NG + (e - J);
            const int r = a.periodic ? row_of(c, nx, 1) : min(max(c, -NG), nx + NG - 1) + NG;
            double v = 0.0;
            if constexpr (BOOK) {
                v = a.U_s[3 * (size_t)r];
            } else {
                const R *ph = a.psi_s + (size_t)r * C2;
                for (int k = lane; k < Q; k += 64) v += (double)ph[k];
#pragma unroll
                for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
                if constexpr (DEV) v += a.ref_sum[0];
            }
            if (lane == 0) next[left ? e : J + rows + (e - J)] = v;
        }
        __syncthreads();
        for (int j = tid; j < rows; j += NT) {
            double nb = 0.0;
            for (int m = 0; m <= 2 * J; ++m) nb = fma(wts[m], next[j + m], nb);
            double eta = 0.25 * a.b * nb;
            if (!(nb > 0.0) || !(eta < 1.0)) {
                atomicOr(a.flag, 1);
                eta = 0.0;  // keep the block finite; the flag reports the failure
            }
            const double cc = chi_set(eta);
            rchi[j] = cc;
            rlnchi[j] = log(cc);
        }
        __syncthreads();
    }

    // ---- phase B.  The cell's divisions are shared: one for chi_SET and d ln chi / d ln n,
    // one for 1/tau, Pr, 1/T and 1/n (the chain of dependent FP64 divisions is the
    // latency of this one-wave phase).
    const double cdt = a.a_L * a.dt;  // RK weight of the right-hand side
    const double idx = 1.0 / a.dx, imu = 1.0 / a.mu_ref;
    for (int i = tid; i < wcount; i += NT) {
        const int j = i + NG;
        const double n = r_n[j], u = r_u[j], T = r_T[j], q = r_q[j];
        const double eta = 0.25 * a.b * n;
#define FD6(f) ((0.75 * ((f)[j + 1] - (f)[j - 1]) - 0.15 * ((f)[j + 2] - (f)[j - 2]) + \
                 ((f)[j + 3] - (f)[j - 3]) * (1.0 / 60.0)) * idx)
        const double dlnn = FD6(r_lnn);
        const double du = FD6(r_u);
        const double dlnT = FD6(r_lnT);
        double chi, dlnchi;
        if constexpr (RET) {
            chi = rchi[j];
            dlnchi = FD6(rlnchi);
        } else {
            // chi = (2 - eta) / (2 (1 - eta)^3), d ln chi / d ln n = eta (5 - 2 eta) /
            // ((1 - eta)(2 - eta))  (Sec. II.A, chain rule from ln n)
            const double om = 1.0 - eta, tw = 2.0 - eta;
            const double d1 = om * om * om, d2 = om * tw;
            const double r1 = 1.0 / (d1 * d2);
            chi = 0.5 * tw * (r1 * d2);
            dlnchi = eta * (5.0 - 2.0 * eta) * (r1 * d1) * dlnn;
        }
#undef FD6
        const double y = a.b * n * chi;
        // mu = (mu_ref sqrt T / chi) dmu, Pr = (2/3) dmu / dpr (Sec. II.B)
        const double cm = (4.0 / 25.0) * (1.0 + 12.0 / M_PI);
        const double cl = (9.0 / 25.0) * (1.0 + 32.0 / (9.0 * M_PI));
        const double dmu = 1.0 + 0.8 * y + cm * y * y;
        const double dpr = a.pr_enskog ? 1.0 + 1.2 * y + cl * y * y : 1.0;
        const double ab = dmu * dpr, nT = n * T;
        const double r2 = 1.0 / (ab * nT);
        const double pr = a.pr_enskog ? (2.0 / 3.0) * dmu * (r2 * dmu * nT) : a.pr;
        const double itau = n * chi * sqrt(T) * imu * (r2 * dpr * nT);  // 1/tau = n T / mu
        const double iT = r2 * ab * n, in = r2 * ab * T;
        if constexpr (CL) csc_s[i] = n * itau;  // scale of the learned closure's output
        // per-cell constants of the march, in four 16-byte groups: three read by every item,
        // the last by the theta items (items that choose phi or theta per lane form the theta
        // terms from the phi ones).  With x2 = xi^2 / T, the J1 bracket is
        // xi (A + C (x2 + e2)) + B (x2 - e1) and the Shakhov factor qc xi (x2 - e0), with
        // (e0, e1, e2) = (3, 1, 1/3) for phi and (1, 1/3, 7/3) for theta, A = d ln chi + 2 d ln n,
        // B = 0.6 du, C = 0.3 d ln T (derivatives in x), qc = (1 - Pr) q / (5 n T^2).
        const double A = dlnchi + 2.0 * dlnn, Bu = 0.6 * du, C = 0.3 * dlnT;
        const double qc = (1.0 - pr) * (0.2 * in) * iT * iT * q;
        R *cv = cellv + i * 16;
        cv[0] = (R)u;
        cv[1] = (R)iT;
        cv[2] = (R)qc;
        cv[3] = (R)C;
        cv[4] = (R)Bu;
        cv[5] = (R)(-y * cdt);                          // J1 prefactor times the RK weight
        cv[6] = (R)(cdt * itau);
        // FP32 storage: a pseudo-random word of (cell, launch) for the stochastic rounding
        if constexpr (DEV)
            reinterpret_cast<unsigned *>(cv)[7] = mix32((unsigned)(i0 + i) * 0x9E3779B1u ^ sd * 0x85EBCA77u);
        else
            cv[7] = R(0);
        cv[8] = (R)(A + C * (1.0 / 3.0));               // phi: A + C e2
        cv[9] = (R)(-3.0 * qc);                         //      -qc e0
        cv[10] = (R)(2.0 * T);                          // theta: 2T
        cv[11] = (R)(DEV ? 2.0 * (T - a.T_ref) : 0.0);  //        2 (T - T_r)
        cv[12] = (R)(A + C * (7.0 / 3.0));              //        A + C e2
        cv[13] = (R)(-Bu * (1.0 / 3.0));                //        -B e1
        cv[14] = R(0);
        cv[15] = R(0);
        if constexpr (BOOK) {
            // exact moments of J1 (eq. j1_expanded): momentum -y n T (dlnchi + 2 dlnn + dlnT),
            // energy u * momentum - y n T du; its mass moment vanishes
            double m1 = -y * n * T * (dlnchi + 2.0 * dlnn + dlnT);
            jm[2 * i] = m1;
            jm[2 * i + 1] = u * m1 - y * n * T * du;
            // U^n of the cell for the RK combination, loaded here, long before its use
            if (a.a_n != 0.0) {
                const double *Un = a.U_n + 3 * (size_t)(i0 + i + NG);
                ucell[3 * W + 3 * i + 0] = Un[0];
                ucell[3 * W + 3 * i + 1] = Un[1];
                ucell[3 * W + 3 * i + 2] = Un[2];
            }
        }
    }
    if constexpr (CL) {
        // the learned closure's inputs of every cell, as its training samples define them:
        // n, u, T, q / (n T^{3/2}), Pxx / (n T) - 1, the gradients of n, u, T, q, Pxx times
        // the local relaxation length sqrt(T) tau over their own scales, E_l and log10 Kn;
        // normalised in FP32 and checked against the training range.  A pass of its own, one
        // gradient at a time (the memory barriers keep the compiler from holding every
        // stencil at once while the march's window is live).
        for (int i = tid; i < wcount; i += NT) {
            const int j = i + NG;
            auto fd6 = [&](const double *f) {
                asm volatile("" ::: "memory");
                return (0.75 * (f[j + 1] - f[j - 1]) - 0.15 * (f[j + 2] - f[j - 2]) +
                        (f[j + 3] - f[j - 3]) * (1.0 / 60.0)) * idx;
            };
            const double n = r_n[j], u = r_u[j], T = r_T[j], q = r_q[j], pxx = r_pxx[j];
            const double nT = n * T, sT = sqrt(T), qs = nT * sT;
            const double lam = sT * n / csc_s[i];  // sqrt(T) tau
            double cx[MLP_IN];
            cx[0] = n; cx[1] = u; cx[2] = T;
            cx[3] = q / qs;
            cx[4] = pxx / nT - 1.0;
            cx[5] = lam * fd6(r_n) / n;
            cx[6] = lam * fd6(r_u) / sT;
            cx[7] = lam * fd6(r_T) / T;
            cx[8] = lam * fd6(r_q) / qs;
            cx[9] = lam * fd6(r_pxx) / nT;
            cx[10] = a.cl_denseness;
            cx[11] = a.cl_log10kn;
            int inside = 1;
            unsigned short *ci = cin_s + i * 16;
            const float *nrm = reinterpret_cast<const float *>(cst_s + CLP);
#pragma unroll
            for (int c = 0; c < MLP_IN; ++c) {
                const float v = ((float)cx[c] - nrm[NRM_IN_MEAN + c]) / nrm[NRM_IN_STD + c];
                if (!(v >= nrm[NRM_LO + c] && v <= nrm[NRM_HI + c])) inside = 0;
                ci[c] = f2bf(v);
            }
#pragma unroll
            for (int c = MLP_IN; c < 16; ++c) ci[c] = 0;
            cok_s[i] = inside;
        }
    }

    // ---- phase B2 (threads after the per-cell items): n c_l, l = 0..N, with
    // c_{l+1} = (u c_l + (T - 1) sqrt(l) c_{l-1}) / sqrt(l + 1), c_0 = 1, c_1 = u, written as
    // c_{l+1} = A_l c_l + B_l c_{l-1}, A_l = u / sqrt(l+1), B_l = (T - 1) sqrt(l / (l+1)).
    // RG lanes per cell split the steps l = 1..N-1 into segments: each lane forms its
    // segment's transfer matrix prod [[A_l, B_l], [1, 0]], a scan over the lanes before it
    // gives the segment's starting pair (c_{l0}, c_{l0-1}), and the lane then runs its
    // segment.  With deviation storage the reference coefficients n_r c_l(u_r, T_r) are
    // subtracted.  Split projection: even orders go to ci[l / 2], odd ones to ci[QH + l / 2].
    {
        const int t = tid - (NT - RG * W);
        if (t >= 0 && t / RG < wcount) {
            const int i = t / RG, g = t - i * RG;
            const int j = i + NG;
            const double n = r_n[j], u = r_u[j], tm1 = r_T[j] - 1.0;
            const int steps = a.N - 1;
            const int l0 = 1 + (g * steps) / RG, l1 = 1 + ((g + 1) * steps) / RG;
            R *ci = cbuf + i * GS;
            auto put = [&](int l, double c) {
                const int o = SPLIT ? (l & 1) * QH + (l >> 1) : l;
                ci[o] = (R)(n * c - (DEV ? cref_s[DEV ? l : 0] : 0.0));
            };
            double s0 = u, s1 = 1.0;  // (c_{l0}, c_{l0 - 1})
            if constexpr (RG > 1) {
                double m00 = 1.0, m01 = 0.0, m10 = 0.0, m11 = 1.0;
#pragma unroll 2
                for (int l = l0; l < l1; ++l) {
                    const double A = u * rec_s[l + 1], B = tm1 * rec_s[QP + l];
                    const double n00 = fma(A, m00, B * m10), n01 = fma(A, m01, B * m11);
                    m10 = m00;
                    m11 = m01;
                    m00 = n00;
                    m01 = n01;
                }
                // the cell's RG lanes are consecutive and RG-aligned inside a DPP row: an
                // inclusive scan of the segment matrices, X_g = M_g ... M_0, by doubling
                // steps (lane g takes X_{g-d} from lane g - d), then s = X_{g-1} (c_1, c_0)
                scan_step<1, RG>(m00, m01, m10, m11, g);
                scan_step<2, RG>(m00, m01, m10, m11, g);
                scan_step<4, RG>(m00, m01, m10, m11, g);
                scan_step<8, RG>(m00, m01, m10, m11, g);
                const double e00 = dpp_f64<DPP_SHR + 1>(m00), e01 = dpp_f64<DPP_SHR + 1>(m01);
                const double e10 = dpp_f64<DPP_SHR + 1>(m10), e11 = dpp_f64<DPP_SHR + 1>(m11);
                if (g > 0) {
                    s0 = fma(e00, u, e01);
                    s1 = fma(e10, u, e11);
                }
            }
            if (g == 0) {
                put(0, 1.0);
                put(1, u);
            }
            double cc = s0, cm = s1;
#pragma unroll 2
            for (int l = l0; l < l1; ++l) {
                const double cn = fma(u * rec_s[l + 1], cc, (tm1 * rec_s[QP + l]) * cm);
                cm = cc;
                cc = cn;
                put(l + 1, cc);
            }
        }
    }
    __syncthreads();

    // ---- phase C: g[i][k] = sum_l c[i][l] Bt[l][k]  (n g, or its deviation).
    // Split form: for the positive nodes k = QH + j, E[i][j] = sum_{l even} c_l Bt[l][k] and
    // O[i][j] = sum_{l odd} c_l Bt[l][k]; then g_k = E + O and g_{Q-1-k} = E - O (phase D).
    // One (16-cell, 16-node, parity) tile per wave (full form: one 16 x 16 tile of g).  The
    // contraction index of a tile is kk KS + ks for lane group kk = lane / 16 at MFMA step ks,
    // so a lane's A values are contiguous in LDS and its B values come from the packed
    // table a.Bt, both read with 16-byte loads:
    //   split: Bp[par][tn][lane][ks] = Bt[2 (kk KS + ks) + par][QH + 16 tn + lane % 16]
    //   full:  Bp[tn][lane][ks] = Bt[kk KS + ks][16 tn + lane % 16]
    {
        typedef typename Acc4<R>::type A4;
        constexpr int KD = SPLIT ? QH : QP;          // contraction length of one tile
        constexpr int TM = W / 16, TN = KD / 16, KS = KD / 4, NP = SPLIT ? 2 : 1;
        constexpr int VB = 16 / (int)sizeof(R);      // values per 16-byte load
        static_assert(KS % VB == 0, "k-steps in whole 16-byte loads");
        const int kk = lane >> 4;
        for (int t = wave; t < TM * TN * NP; t += NWAVE) {
            const int par = t % NP, tt = t / NP;
            const int tm = tt / TN, tn = tt - tm * TN;
            const int row = tm * 16 + (lane & 15), col = tn * 16 + (lane & 15);
            const float4 *ap = reinterpret_cast<const float4 *>(cbuf + row * GS + par * QH + kk * KS);
            const float4 *bp = reinterpret_cast<const float4 *>(
                a.Bt + (((size_t)par * TN + tn) * 64 + lane) * KS);
            A4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = R(0);
#pragma unroll
            for (int x = 0; x < KS / VB; ++x) {
                const float4 av4 = ap[x], bv4 = bp[x];
                const R *av = reinterpret_cast<const R *>(&av4);
                const R *bv = reinterpret_cast<const R *>(&bv4);
#pragma unroll
                for (int j = 0; j < VB; ++j) acc = mfma16x16x4(av[j], bv[j], acc);
            }
            // output lane layout (measured): FP32 row 4 (l / 16) + r, FP64 row l / 16 + 4 r;
            // column l % 16 for both
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int orow = sizeof(R) == 4 ? 4 * kk + r : kk + 4 * r;
                gbuf[(tm * 16 + orow) * GS + par * QH + col] = acc[r];
            }
        }
    }
    __syncthreads();

    // ---- phase L (CL): the learned closure's correction of the tile's cells (its
    // activation tiles take the coefficient buffer, free since phase C)
    if constexpr (CL) {
        closure_tile<R, Q, W, NWAVE>(a, cin_s, csc_s, cok_s, cst_s, corr_s,
                                     reinterpret_cast<unsigned short *>(cbuf), wcount, wave, lane);
        __syncthreads();
    }

    // ---- phase D (the threads of a padded block beyond the 2 S Q items have ds >= S)
    __builtin_amdgcn_s_setprio(0);
    if (!PADDED || ds < S) {
        // FP32: psi^n at this item's cells (stages 2 and 3), loaded before the march: its
        // stores may alias these addresses (the last stage writes over psi^n), so loads
        // issued inside the march could not be moved ahead of the stores before them.  (FP64
        // keeps the loads in the march: the registers would spill.)
        // One uniform branch around branch-free loads (cells past a partial tile read the
        // tile's last cell and are not stored), so that each cell waits for its own load only.
        constexpr bool PRE = sizeof(R) == 4;
        R pn[PRE ? L : 1];
        if constexpr (PRE) {
            const R *const nrow = a.psi_n + (size_t)(i0 + NG) * C2 + dc;
            if (a.a_n != 0.0) {
#pragma unroll
                for (int m = 0; m < L; ++m) pn[m] = nrow[(size_t)min(ib + m, wcount - 1) * C2];
            } else {
#pragma unroll
                for (int m = 0; m < L; ++m) pn[m] = R(0);
            }
        }
        const R pk = (R)pk_s[k];
        const R gref = DEV ? (R)gref_s[k] : R(0);  // n_r g_k(u_r, T_r)
        const int kp = neg ? QH - 1 - k : k - QH;   // positive node of the pair (E, O index)
        const R pidx = (R)(a.a_L * a.dt / (6.0 * a.dx)) * pk;  // RK weight x p_k / (6 dx)
        const R pk6 = pk / R(6);                    // flux = interpolant x p_k / 6
        const R a_n = (R)a.a_n;
        const bool has_n = a.a_n != 0.0;
        const int mlim = wcount - ib;               // cells of this strip inside the tile
        R *const outp = a.psi_out + (size_t)(i0 + ib + NG) * C2 + dc;
        const R *const inp = a.psi_n + (size_t)(i0 + ib + NG) * C2 + dc;
        const R *const cvb = cellv + ib * 16;       // per-cell constants of the strip
        const R *const gbb = gbuf + ib * GS;        // equilibrium rows of the strip
        R *const fxb = cbuf + ib * FS + dc;         // bookkeeping: flux rows of the strip
        // the learned closure's correction at this item's cells (phi items only): fused,
        // from LDS; separate, from its [nx][Q] buffer
        const R *const corr = CL ? corr_s + ib * Q + k : a.corr ? a.corr + (size_t)(i0 + ib) * Q + k : nullptr;
        // FP32 storage: pseudo-random word of (column, launch); with the word of the cell it
        // gives the byte that dithers this item's store in that cell
        const unsigned hc = DEV ? mix32((unsigned)dc * 0x632BE5ABu ^ sd * 0xC2B2AE35u) : 0u;
        // The march for one velocity sign (NEGC) and one distribution (THC: 0 phi, 1 theta,
        // 2 chosen per lane by isth).  Every interface is formed by the same sequence of
        // shift() operations (the first one of a strip from five shifts of a zero state), so
        // its value does not depend on where a strip or a tile starts.  With bookkeeping,
        // interface j (0..W) of a column is stored by exactly one strip; rows past the tile's
        // last interface (partial tiles) are never read.
        auto march = [&](auto negc, auto thc) {
            constexpr bool NEGC = decltype(negc)::value;
            constexpr int THC = decltype(thc)::value;
            const bool th = THC == 2 ? isth : THC == 1;
            // phi: psi_S = n g (1 + sh), theta: psi_S = 2 T n g (1 + sh), sh = qc xi (x2 - e0);
            // per-lane choice (THC = 2): the e-terms from the phi constants, A + C e2 =
            // (A + C/3) + C (e2 - 1/3), -B e1 = B (-e1), -qc e0 = qc (-e0)
            const R de2 = th ? R(2) : R(0);
            const R ne1 = th ? R(-1) / R(3) : R(-1);
            const R ne0 = th ? R(-1) : R(-3);
            // one cell of the march: I_in, I_out are 6 x the interpolants at the upwind and
            // downwind interfaces; the flux difference F_{i+1/2} - F_{i-1/2} is
            // p (I_out - I_in) / 6 for p > 0 and p (I_in - I_out) / 6 for p < 0
            // the LDS values of cell m: its constants and the equilibrium (E and O half sums,
            // or g).  FP32 reads them before the cell's interface is interpolated, so that the
            // read latency overlaps that work (FP64 after it: its registers would not hold
            // both; so does the moment fix-up, which spilled at Q = 64), and reads only the
            // constants the distribution uses (phi: 0-9, theta: 0-7 and 10-13; per-lane
            // choice: 0-11), so that no read lands in the registers of an unused value, which
            // the next read could take over.
            constexpr bool EARLY = sizeof(R) == 4 && !FIX;
            constexpr int NG4 = THC == 1 ? 4 : 3;
            struct CellIn { R cv[16]; R e, o; };
            auto fetch = [&](const int m) {
                CellIn ci;
                if constexpr (sizeof(R) == 4) {
                    const floatx4 *cq = reinterpret_cast<const floatx4 *>(cvb + m * 16);
                    const floatx2 *ch = reinterpret_cast<const floatx2 *>(cvb + m * 16);
#pragma unroll
                    for (int q4 = 0; q4 < 2; ++q4) {
                        const floatx4 x = cq[q4];
                        ci.cv[4 * q4] = x.x; ci.cv[4 * q4 + 1] = x.y;
                        ci.cv[4 * q4 + 2] = x.z; ci.cv[4 * q4 + 3] = x.w;
                    }
                    if constexpr (THC == 0) {
                        const floatx2 x = ch[4];
                        ci.cv[8] = x.x; ci.cv[9] = x.y;
                    } else if constexpr (THC == 1) {
                        const floatx2 x = ch[5], y = ch[6];
                        ci.cv[10] = x.x; ci.cv[11] = x.y; ci.cv[12] = y.x; ci.cv[13] = y.y;
                    } else {
                        const floatx4 x = cq[2];
                        ci.cv[8] = x.x; ci.cv[9] = x.y; ci.cv[10] = x.z; ci.cv[11] = x.w;
                    }
                } else {
#pragma unroll
                    for (int t = 0; t < 4 * NG4; ++t) ci.cv[t] = cvb[m * 16 + t];
                }
                if constexpr (SPLIT) {
                    ci.e = gbb[m * GS + kp];
                    ci.o = gbb[m * GS + QH + kp];
                } else {
                    ci.e = gbb[m * GS + k];
                    ci.o = R(0);
                }
                return ci;
            };
            auto cell = [&](const int m, const CellIn &ci, const R f3, const R I_in, const R I_out) {
                const R *const cv = ci.cv;
                const R u = cv[0], iT = cv[1], qc = cv[2], C = cv[3], Bu = cv[4];
                const R myw = cv[5], itw = cv[6];
                R Ap, Bp, Qp;                           // A + C e2, -B e1, -qc e0
                if constexpr (THC == 0) {
                    Ap = cv[8]; Bp = -Bu; Qp = cv[9];
                } else if constexpr (THC == 1) {
                    Ap = cv[12]; Bp = cv[13]; Qp = -qc;
                } else {
                    Ap = fma(C, de2, cv[8]); Bp = Bu * ne1; Qp = qc * ne0;
                }
                // n g_k, or n g_k - n_r g_k^r
                const R dg = SPLIT ? (NEGC ? ci.e - ci.o : ci.e + ci.o) : ci.e;
                const R xi = pk - u;
                const R x2 = xi * xi * iT;
                const R sh = xi * fma(qc, x2, Qp);      // qc xi (x2 - e0)
                // (1 or 2T) n g_k and the Shakhov target (or its deviation from psi_ref:
                // theta takes 2T dg + 2 (T - T_r) n_r g^r, which keeps the deviation's precision)
                R mng, psiS;
                if constexpr (THC == 2) {
                    const R mth = th ? cv[10] : R(1);   // 1 (phi) or 2T (theta)
                    const R dth = th ? cv[11] : R(0);   // 0 (phi) or 2 (T - T_r) (theta)
                    mng = mth * (dg + gref);
                    psiS = fma(mng, sh, fma(mth, dg, dth * gref));
                } else if constexpr (THC == 1) {
                    mng = cv[10] * (dg + gref);
                    psiS = fma(mng, sh, fma(cv[10], dg, cv[11] * gref));
                } else {
                    mng = dg + gref;
                    psiS = fma(mng, sh, dg);
                }
                const R br = fma(xi, fma(C, x2, Ap), fma(Bu, x2, Bp));
                const R dI = NEGC ? I_in - I_out : I_out - I_in;
                // a_n + a_s = 1 in every stage: psi^(s) + a_n (psi^n - psi^(s)) keeps the
                // combination free of the rounding of a_n and a_s
                if constexpr (DEV) {
                    // FP32 storage: out = f3 + D is rounded stochastically.  A dither uniform
                    // on (-1/2, 1/2) ulp of the result (a pseudo-random byte) is added to the
                    // increment before the round-to-nearest sum, so the stored value is f3 + D
                    // in expectation.  Deterministic rounding would give each slowly varying
                    // value the same rounding error step after step, and those errors would
                    // add up over long runs.  Stage 1 loaded pn = 0 (a_n = 0 adds a zero).
                    R D = -pidx * dI - (f3 - psiS) * itw + myw * br * mng + a_n * (pn[m] - f3);
                    if (THC != 1 && !th && corr && m < mlim) D += (R)cdt * corr[(size_t)m * Q];
                    const unsigned eb = __builtin_elementwise_sub_sat(
                        __float_as_uint(f3 + D) & 0x7f800000u, 31u << 23);   // ulp / 256
                    const float byte = (float)((__float_as_uint(cv[7]) ^ hc) & 255u);
                    const R out = f3 + fma(__uint_as_float(eb), byte - 127.5f, D);
                    if (m < mlim) outp[(size_t)m * C2] = out;
                } else {
                    R out = f3 - pidx * dI - (f3 - psiS) * itw + myw * br * mng;
                    if (m < mlim) {
                        if (THC != 1 && !th && corr) out += (R)cdt * corr[(size_t)m * Q];
                        if (has_n) out += a_n * (inp[(size_t)m * C2] - f3);
                        outp[(size_t)m * C2] = out;
                    }
                }
            };
            WenoMarch<R> wm;
            wm.zero();
            if constexpr (NEGC) {
                // right to left: the interface i-1/2 of cell i has the upwind stencil
                // (f_{i+2}, f_{i+1}, f_i, f_{i-1}, f_{i-2}); win[x] = f_{ib-3+x}
#pragma unroll
                for (int x = 0; x < 5; ++x) wm.shift(win[L + 5 - x]);
                R Iprev = wm.interp6();                 // interface ib + L - 1/2
                if constexpr (BOOK)
                    if (ds == S - 1) fxb[L * FS] = Iprev * pk6;
#pragma unroll
                for (int mm = 0; mm < L; ++mm) {
                    const int m = L - 1 - mm;           // cell ib + m
                    CellIn ci;
                    if constexpr (EARLY) ci = fetch(m);
                    wm.shift(win[m + 1]);                // f_{i-2} (win[x] = f_{ib-3+x})
                    const R I = wm.interp6();            // interface ib + m - 1/2
                    if constexpr (BOOK) fxb[m * FS] = I * pk6;
                    if constexpr (!EARLY) ci = fetch(m);
                    cell(m, ci, win[m + 3], Iprev, I);
                    Iprev = I;
                }
            } else {
                // left to right: the interface i+1/2 of cell i has (f_{i-2}, ..., f_{i+2})
#pragma unroll
                for (int x = 0; x < 5; ++x) wm.shift(win[x]);
                R Iprev = wm.interp6();                 // interface ib - 1/2
                if constexpr (BOOK)
                    if (ds == 0) fxb[0] = Iprev * pk6;
#pragma unroll
                for (int m = 0; m < L; ++m) {
                    CellIn ci;
                    if constexpr (EARLY) ci = fetch(m);
                    wm.shift(win[m + 5]);                // f_{i+2}
                    const R I = wm.interp6();            // interface ib + m + 1/2
                    if constexpr (BOOK) fxb[(m + 1) * FS] = I * pk6;
                    if constexpr (!EARLY) ci = fetch(m);
                    cell(m, ci, win[m + 3], Iprev, I);
                    Iprev = I;
                }
            }
        };
        using T_ = std::integral_constant<bool, true>;
        using F_ = std::integral_constant<bool, false>;
        using P0 = std::integral_constant<int, 0>;
        using P1 = std::integral_constant<int, 1>;
        using P2 = std::integral_constant<int, 2>;
        if constexpr (THW) {
            if (neg_w) {
                if (th_w) march(T_{}, P1{});
                else march(T_{}, P0{});
            } else {
                if (th_w) march(F_{}, P1{});
                else march(F_{}, P0{});
            }
        } else {
            if (neg_w) march(T_{}, P2{});
            else march(F_{}, P2{});
        }
    }

    __builtin_amdgcn_s_setprio(2);

    // ---- phase E (bookkeeping): per interface j, G_j = sum over columns of the stored flux
    // values times (1, p, p^2/2) for phi and (0, 0, 1/2) for theta, in FP64; 8 lanes per
    // interface, each summing every 8th column, then 3 exchange steps.  Only the threads of
    // the W + 1 interfaces take part (the 8 lanes of an interface are active together).
    if constexpr (BOOK) {
        __syncthreads();
        {
            const int part = tid & 7;
            for (int j = tid >> 3; j <= wcount; j += NT / 8) {
                double v0 = 0.0, v1 = 0.0, v2;
                if constexpr (Q % 8 == 0) {
                    // lane `part` takes the phi columns part + 8 m (m < Q/8), then the theta
                    // columns, which carry energy only
                    double e = 0.0;
#pragma unroll
                    for (int m = 0; m < Q / 8; ++m) {
                        const int c = part + 8 * m;
                        const double F = (double)cbuf[j * FS + c];
                        const double pF = pk_s[c] * F;
                        v0 += F;
                        v1 += pF;
                        e = fma(pk_s[c], pF, e);
                    }
#pragma unroll
                    for (int m = Q / 8; m < C2 / 8; ++m) e += (double)cbuf[j * FS + part + 8 * m];
                    v2 = 0.5 * e;
                } else {
                    v2 = 0.0;
                    for (int c = part; c < C2; c += 8) {
                        const double F = (double)cbuf[j * FS + c];
                        const bool isphi = c < Q;
                        const double pk = pk_s[isphi ? c : c - Q];
                        const double Fp = isphi ? F : 0.0;
                        v0 += Fp;
                        v1 = fma(pk, Fp, v1);
                        v2 = fma(isphi ? 0.5 * pk * pk : 0.5, F, v2);
                    }
                }
                v0 = sum8_dpp(v0);
                v1 = sum8_dpp(v1);
                v2 = sum8_dpp(v2);
                if (part == 0) {
                    gsum[j * 3 + 0] = v0;
                    gsum[j * 3 + 1] = v1;
                    gsum[j * 3 + 2] = v2;
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < wcount; i += NT) {
            const double idx = 1.0 / a.dx;
            const size_t r = (size_t)(i0 + i + NG);
            const double *Us = ucell + 3 * i;
            const double *Un = ucell + 3 * W + 3 * i;
            double d[3];
            d[0] = -(gsum[(i + 1) * 3 + 0] - gsum[i * 3 + 0]) * idx;
            d[1] = -(gsum[(i + 1) * 3 + 1] - gsum[i * 3 + 1]) * idx + jm[2 * i];
            d[2] = -(gsum[(i + 1) * 3 + 2] - gsum[i * 3 + 2]) * idx + jm[2 * i + 1];
            double outv[3];
            for (int m = 0; m < 3; ++m) {
                double v = Us[m] + a.a_L * a.dt * d[m];
                if (a.a_n != 0.0) v += a.a_n * (Un[m] - Us[m]);
                outv[m] = v;
            }
            for (int m = 0; m < 3; ++m) a.U_out[3 * r + m] = outv[m];
        }
    }
}

// One launch of a stage over one problem: block b handles the tile of cells [b W, b W + W).
// RET: chi and d ln chi from the ball-averaged density (chi_RET-FM, phase R, with dynamic
// LDS) instead of chi_SET of the cell; a separate instantiation, so the chi_SET kernel
// carries none of it.  CL: the learned closure evaluated inside the stage (phase L), also
// an instantiation of its own (Q <= 16).
template <typename R, int Q, int MODE, bool RET, bool CL = false>
__global__ __launch_bounds__((Geometry<R, Q>::NT))
__attribute__((amdgpu_waves_per_eu(CL ? Geometry<R, Q>::WVCL : Geometry<R, Q>::WV))) void k_stage(StageArgs<R> a)
{
    stage_tile<R, Q, Geometry<R, Q>::S, Geometry<R, Q>::L, MODE, RET, CL>(a, blockIdx.x);
}

// Batched form: per-instance description (device array) and the (instance, tile) items of
// one group of instances sharing Q and the tile shape; block b takes item b, so one launch
// covers the whole group.
struct InstDesc {
    void *psi[3];
    double *U[3];
    const double *p, *w, *cref, *gref, *rec;
    const void *Bt;
    int *flag;
    int nx, N, periodic, pr_enskog;
    double dx, dt, b, mu_ref, pr, T_ref;
    double ref_sum[6];
    const double *fm_w;  // chi_RET-FM weights (RET kernels), half-width fm_J
    int fm_J;
};

struct BatchStage {
    const InstDesc *inst;
    const int2 *items;   // (instance, tile)
    int nitems;
    int s_in, s_out;     // levels read (stage input) and written
    double a_n, a_s, a_L;
    unsigned seed;       // stochastic rounding stream (see StageArgs)
    const unsigned *seed_base;
};

template <typename R, int Q, int S_, int L_, int MODE, bool RET>
__global__ __launch_bounds__((Geometry<R, Q, S_, L_>::NT))
__attribute__((amdgpu_waves_per_eu(Geometry<R, Q, S_, L_>::WV))) void k_stage_batch(BatchStage bs)
{
    {
        const int item = blockIdx.x;  // one (instance, tile) item per block
        if (item >= bs.nitems) return;
        const int2 it = bs.items[item];
        const InstDesc &d = bs.inst[it.x];
        StageArgs<R> a;
        a.psi_s = (const R *)d.psi[bs.s_in];
        a.psi_n = (const R *)d.psi[0];
        a.psi_out = (R *)d.psi[bs.s_out];
        a.U_s = d.U[bs.s_in];
        a.U_n = d.U[0];
        a.U_out = d.U[bs.s_out];
        a.p = d.p;
        a.Bt = (const R *)d.Bt;
        a.cref = d.cref;
        a.gref = d.gref;
        a.rec = d.rec;
        a.w = d.w;
        a.flag = d.flag;
        a.nx = d.nx;
        a.N = d.N;
        a.periodic = d.periodic;
        a.pr_enskog = d.pr_enskog;
        a.dx = d.dx;
        a.dt = d.dt;
        a.b = d.b;
        a.mu_ref = d.mu_ref;
        a.pr = d.pr;
        a.a_n = bs.a_n;
        a.a_s = bs.a_s;
        a.a_L = bs.a_L;
        a.T_ref = d.T_ref;
        for (int m = 0; m < 6; ++m) a.ref_sum[m] = d.ref_sum[m];
        a.corr = nullptr;
        a.fm_w = RET ? d.fm_w : nullptr;
        a.fm_J = d.fm_J;
        a.seed = bs.seed;
        a.seed_base = bs.seed_base;
        stage_tile<R, Q, S_, L_, MODE, RET>(a, it.y);
    }
}

// Base of the stochastic rounding stream for the next replay of a captured graph.
__global__ void k_set_seed(unsigned *base, unsigned value)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *base = value;
}

// --------------------------------------------------------------------------------------
// Equilibrium initialisation of rows [0, rows): phi_k = n g_k(u,T), theta_k = 2 T n g_k,
// g_k = sum_l Bt[l][k] c_l(u, T) in FP64 (QP-strided table), minus the per-column reference
// (zero in FP64 storage).  One thread per (row, node).  With U != NULL also the conserved
// densities (n, n u, (n u^2 + 3 n T)/2) of every row.
// --------------------------------------------------------------------------------------
template <typename R>
__global__ void k_init_equilibrium(R *psi, double *U, const double *nrow, const double *urow,
                                   const double *Trow, const double *Bt, const double *sq,
                                   const double *rsq, const double *ref, int rows, int Q, int QP,
                                   int N)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // rows * Q may pass 2^31
    if (idx >= (size_t)rows * Q) return;
    const int r = (int)(idx / Q), k = (int)(idx - (size_t)r * Q);
    double n = nrow[r], u = urow[r], T = Trow[r];
    double cm = 1.0, cc = u;
    double g = Bt[k] * cm;
    if (N >= 1) g += Bt[QP + k] * cc;
    for (int l = 1; l < N; ++l) {
        double cn = (u * cc + (T - 1.0) * sq[l] * cm) * rsq[l + 1];
        cm = cc;
        cc = cn;
        g += Bt[(l + 1) * QP + k] * cc;
    }
    psi[(size_t)r * 2 * Q + k] = (R)(n * g - ref[k]);
    psi[(size_t)r * 2 * Q + Q + k] = (R)(2.0 * T * n * g - ref[Q + k]);
    if (U && k == 0) {
        U[3 * (size_t)r + 0] = n;
        U[3 * (size_t)r + 1] = n * u;
        U[3 * (size_t)r + 2] = 0.5 * (n * u * u + 3.0 * n * T);
    }
}

// Conserved densities of every row from the stored distributions plus reference (FP64 sums).
template <typename R>
__global__ void k_conserved_from_psi(const R *psi, const double *ref, double *U, const double *p,
                                     int rows, int Q)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    const R *ph = psi + (size_t)r * 2 * Q;
    double n = 0, j = 0, e = 0;
    for (int k = 0; k < Q; ++k) {
        double v = (double)ph[k] + ref[k];
        n += v;
        j += p[k] * v;
        e += 0.5 * (p[k] * p[k] * v + (double)ph[Q + k] + ref[Q + k]);
    }
    U[3 * (size_t)r] = n;
    U[3 * (size_t)r + 1] = j;
    U[3 * (size_t)r + 2] = e;
}

// Per interior cell: n, u, T, q_x, P_xx (Sec. II.D) in FP64, two passes over the nodes, and
// the conserved densities (n, n u, E).  With U != NULL (bookkeeping) n, u, T and the
// conserved densities are the tracked ones; q_x and P_xx use that u.  `ref` is added to the
// stored values (deviation storage; zero for FP64).
//
// 16 lanes per cell (MOM_LANES), so a wave reads four rows as 64-byte segments: lane m
// takes the nodes m, m + 16, ... of phi and theta, and each pass ends with 4 exchange steps
// inside the 16-lane group.  The second pass re-reads the row from cache.
constexpr int MOM_LANES = 16;

__device__ inline double sum16(double v)
{
#pragma unroll
    for (int m = MOM_LANES / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, MOM_LANES);
    return v;
}

template <typename R>
__global__ void k_moments(const R *psi, const double *ref, const double *U, const double *p,
                          int nx, int Q, double *out_n, double *out_u, double *out_T,
                          double *out_q, double *out_pxx, double *out_cons)
{
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t i = gid / MOM_LANES;           // one cell per 16-lane group
    const int part = (int)(gid % MOM_LANES);
    // every lane of a group shares i, so a group is live or idle as a whole; idle groups
    // still run the exchanges (on zeros) and store nothing
    const bool live = i < (size_t)nx;
    const R *ph = psi + (live ? i + NG : (size_t)NG) * 2 * Q;
    const R *th = ph + Q;
    double n = 0, j = 0, e2 = 0;
    if (live)
        for (int k = part; k < Q; k += MOM_LANES) {
            const double v = (double)ph[k] + ref[k];
            n += v;
            j += p[k] * v;
            e2 += 0.5 * (p[k] * p[k] * v + (double)th[k] + ref[Q + k]);
        }
    n = sum16(n);
    j = sum16(j);
    e2 = sum16(e2);
    if (U && live) {
        const double *Ui = U + 3 * (i + NG);
        n = Ui[0];
        j = Ui[1];
        e2 = Ui[2];
    }
    const double u = live ? j / n : 0.0;
    double pxx = 0, e = 0, q = 0;
    if (live)
        for (int k = part; k < Q; k += MOM_LANES) {
            const double xi = p[k] - u;
            const double vp = (double)ph[k] + ref[k], vt = (double)th[k] + ref[Q + k];
            const double ek = 0.5 * xi * xi * vp + 0.5 * vt;
            pxx += xi * xi * vp;
            e += ek;
            q += xi * ek;
        }
    pxx = sum16(pxx);
    e = sum16(e);
    q = sum16(q);
    if (live && part == 0) {
        out_n[i] = n;
        out_u[i] = u;
        out_T[i] = U ? (2.0 * e2 / n - u * u) / 3.0 : e / (1.5 * n);
        out_q[i] = q;
        out_pxx[i] = pxx;
        out_cons[3 * i + 0] = n;
        out_cons[3 * i + 1] = j;
        out_cons[3 * i + 2] = e2;
    }
}

}  // namespace elb
