// C ABI of the FDLB solver (include/elb.h): context set-up, workspace layout and the
// launch sequence of the RK3 step on gfx950.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/elb.h"
#include "elb_kernels.h"
#include "host_math.h"

using namespace elb;

namespace {

const int kSupportedQ[] = {8, 12, 16, 24, 32, 48, 64, 96};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t p, btd, btf, sq, rsq, rec, cref, gref, ref, flag, psi[3], U[3], rows, out, cons, total;
};

int padded_q(int q) { return (q + 15) / 16 * 16; }

int elem_size(int precision) { return precision == ELB_FP64 ? 8 : 4; }

Layout make_layout(int nx, int Q, int N, int precision)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align256(o + bytes); return at; };
    L.p = take(sizeof(double) * Q);
    const int QP = padded_q(Q);
    (void)N;
    L.btd = take(sizeof(double) * (size_t)QP * QP);
    L.btf = take(sizeof(float) * (size_t)QP * QP);
    L.sq = take(sizeof(double) * (QP + 2));
    L.rsq = take(sizeof(double) * (QP + 2));
    L.rec = take(sizeof(double) * 2 * QP);
    L.cref = take(sizeof(double) * QP);
    L.gref = take(sizeof(double) * Q);
    L.ref = take(sizeof(double) * 2 * Q);
    L.flag = take(sizeof(int) * 4);
    size_t lvl = (size_t)(nx + 2 * NG) * 2 * Q * elem_size(precision);
    for (int s = 0; s < 3; ++s) L.psi[s] = take(lvl);
    size_t ul = precision == ELB_FP32_MIXED ? sizeof(double) * 3 * (size_t)(nx + 2 * NG) : 0;
    for (int s = 0; s < 3; ++s) L.U[s] = take(ul);
    L.rows = take(sizeof(double) * 3 * (size_t)(nx + 2 * NG));
    L.out = take(sizeof(double) * 5 * (size_t)nx);
    L.cons = take(sizeof(double) * 3 * (size_t)nx);
    L.total = o;
    return L;
}

bool q_supported(int q)
{
    for (int v : kSupportedQ)
        if (v == q) return true;
    return false;
}

}  // namespace

struct elb_ctx {
    elb_params P;
    int Q = 0, N = 0;
    double dx = 0, dt = 0, b = 0, mu_ref = 0, eta0 = 0, chi0 = 0;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    Layout L{};
    std::vector<double> p, w, Btd;
    // deviation storage (FP32): reference state and its per-column distribution
    double n_ref = 0, u_ref = 0, T_ref = 1;
    std::vector<double> ref;     // phi_ref (Q) then theta_ref (Q); zero for FP64 storage
    double ref_sum[6] = {0, 0, 0, 0, 0, 0};
    bool has_state = false;
    int64_t steps = 0;
    std::string err;

    template <typename T>
    T *dev(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

int fail(elb_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

int hip_check(elb_ctx *c, hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(c, ELB_EHIP, "%s: %s", what, hipGetErrorString(e));
    return ELB_OK;
}

// Validates p and fills the derived quantities; returns ELB_OK or an error code with a
// message in *msg.
int derive(const elb_params *p, int *N, double *dx, double *dt, double *b, double *mu_ref,
           double *eta0, double *chi0, std::vector<double> *nodes, std::string *msg)
{
    if (!p) { *msg = "params is NULL"; return ELB_EINVAL; }
    if (p->nx < 8) { *msg = "nx must be >= 8"; return ELB_EINVAL; }
    if (p->q < 7) { *msg = "q must be >= 7 (Shakhov needs moments up to order 6)"; return ELB_EINVAL; }
    if (!q_supported(p->q)) { *msg = "q not among the compiled values (elb_supported_q)"; return ELB_EUNSUPPORTED; }
    int n = p->n_herm == 0 ? p->q - 1 : p->n_herm;
    if (n < 6 || n > p->q - 1) { *msg = "n_herm must be 0 or in [6, q-1]"; return ELB_EINVAL; }
    if (!(p->length > 0) || !std::isfinite(p->length) || !std::isfinite(p->x0)) { *msg = "length must be finite and > 0"; return ELB_EINVAL; }
    if (!(p->denseness >= 0) || !std::isfinite(p->denseness)) { *msg = "denseness must be finite and >= 0"; return ELB_EINVAL; }
    if (!(p->kn > 0) || !(p->kn_length > 0) || !(p->n_ref > 0) || !std::isfinite(p->kn) ||
        !std::isfinite(p->kn_length) || !std::isfinite(p->n_ref)) { *msg = "kn, kn_length, n_ref must be finite and > 0"; return ELB_EINVAL; }
    // the contact value diverges at eta = 1; E_l(eta=0.49) ~ 127
    if (p->denseness > 100.0) { *msg = "denseness above the range of chi_SET used here"; return ELB_EINVAL; }
    if (p->pr_mode != ELB_PR_CONST && p->pr_mode != ELB_PR_ENSKOG) { *msg = "bad pr_mode"; return ELB_EINVAL; }
    if (p->pr_mode == ELB_PR_CONST && !(p->pr > 0 && p->pr <= 10)) { *msg = "pr must be in (0, 10]"; return ELB_EINVAL; }
    if (p->bc != ELB_BC_PERIODIC && p->bc != ELB_BC_EQUILIBRIUM) { *msg = "bad bc"; return ELB_EINVAL; }
    if (p->precision != ELB_FP64 && p->precision != ELB_FP32 && p->precision != ELB_FP32_MIXED) { *msg = "bad precision"; return ELB_EINVAL; }
    if (p->bc == ELB_BC_EQUILIBRIUM) {
        const double *g[2] = {p->ghost_left, p->ghost_right};
        for (auto s : g)
            if (!(s[0] > 0) || !(s[2] > 0) || !std::isfinite(s[0]) || !std::isfinite(s[1]) || !std::isfinite(s[2])) {
                *msg = "ghost states need finite n > 0, T > 0";
                return ELB_EINVAL;
            }
    }
    std::vector<double> pk(p->q), wk(p->q);
    if (gauss_hermite(p->q, pk.data(), wk.data()) != 0) { *msg = "quadrature failed"; return ELB_EINVAL; }
    double pmax = pk.back();
    *N = n;
    *dx = p->length / p->nx;
    if (p->dt > 0) {
        if (!std::isfinite(p->dt)) { *msg = "dt must be finite"; return ELB_EINVAL; }
        *dt = p->dt;
    } else {
        if (!(p->cfl > 0 && p->cfl <= 1.0)) { *msg = "cfl must be in (0, 1] when dt <= 0"; return ELB_EINVAL; }
        *dt = p->cfl * (*dx) / pmax;
    }
    if (*dt * pmax / *dx > 1.0 + 1e-12) { *msg = "dt violates CFL <= 1 for the largest node"; return ELB_EINVAL; }
    map_units(p->denseness, p->kn, p->kn_length, p->n_ref, b, mu_ref, eta0, chi0);
    if (nodes) *nodes = pk;
    return ELB_OK;
}

double host_tau(const elb_ctx *c, double n, double T)
{
    double eta = 0.25 * c->b * n;
    double chi = chi_set(eta);
    double y = c->b * n * chi;
    const double cm = (4.0 / 25.0) * (1.0 + 12.0 / M_PI);
    return c->mu_ref * (1.0 + 0.8 * y + cm * y * y) / (n * chi * std::sqrt(T));
}

template <typename R, int Q, int MODE>
void launch_stage_t(const elb_ctx *c, int s_in, int s_out, double an, double as, double aL)
{
    using G = Geometry<R, Q>;
    StageArgs<R> a{};
    a.psi_s = c->dev<R>(c->L.psi[s_in]);
    a.psi_n = c->dev<R>(c->L.psi[0]);
    a.psi_out = c->dev<R>(c->L.psi[s_out]);
    a.U_s = c->dev<double>(c->L.U[s_in]);
    a.U_n = c->dev<double>(c->L.U[0]);
    a.U_out = c->dev<double>(c->L.U[s_out]);
    a.p = c->dev<double>(c->L.p);
    a.Bt = (sizeof(R) == 8) ? (const R *)c->dev<double>(c->L.btd) : (const R *)c->dev<float>(c->L.btf);
    a.cref = c->dev<double>(c->L.cref);
    a.gref = c->dev<double>(c->L.gref);
    a.rec = c->dev<double>(c->L.rec);
    a.flag = c->dev<int>(c->L.flag);
    a.nx = c->P.nx;
    a.N = c->N;
    a.periodic = c->P.bc == ELB_BC_PERIODIC;
    a.pr_enskog = c->P.pr_mode == ELB_PR_ENSKOG;
    a.dx = c->dx;
    a.dt = c->dt;
    a.b = c->b;
    a.mu_ref = c->mu_ref;
    a.pr = c->P.pr;
    a.a_n = an;
    a.a_s = as;
    a.a_L = aL;
    a.T_ref = c->T_ref;
    for (int m = 0; m < 6; ++m) a.ref_sum[m] = c->ref_sum[m];
    int blocks = (c->P.nx + G::W - 1) / G::W;
    hipLaunchKernelGGL((k_stage<R, Q, MODE>), dim3(blocks), dim3(G::NT), 0, c->stream, a);
}

template <int Q>
void launch_stage_q(const elb_ctx *c, int s_in, int s_out, double an, double as, double aL)
{
    switch (c->P.precision) {
        case ELB_FP64: launch_stage_t<double, Q, MODE_FP64>(c, s_in, s_out, an, as, aL); break;
        case ELB_FP32: launch_stage_t<float, Q, MODE_FP32>(c, s_in, s_out, an, as, aL); break;
        default: launch_stage_t<float, Q, MODE_FP32_MIXED>(c, s_in, s_out, an, as, aL); break;
    }
}

void launch_stage(const elb_ctx *c, int s_in, int s_out, double an, double as, double aL)
{
    switch (c->Q) {
        case 8: launch_stage_q<8>(c, s_in, s_out, an, as, aL); break;
        case 12: launch_stage_q<12>(c, s_in, s_out, an, as, aL); break;
        case 16: launch_stage_q<16>(c, s_in, s_out, an, as, aL); break;
        case 24: launch_stage_q<24>(c, s_in, s_out, an, as, aL); break;
        case 32: launch_stage_q<32>(c, s_in, s_out, an, as, aL); break;
        case 48: launch_stage_q<48>(c, s_in, s_out, an, as, aL); break;
        case 64: launch_stage_q<64>(c, s_in, s_out, an, as, aL); break;
        case 96: launch_stage_q<96>(c, s_in, s_out, an, as, aL); break;
        default: break;
    }
}

// Reference equilibrium of the deviation storage (FP32 modes): the mean state (n_r, u_r,
// T_r) of the given cells; phi_ref_k = n_r g_k(u_r, T_r), theta_ref_k = 2 T_r phi_ref_k, the
// coefficients n_r c_l(u_r, T_r) and the FP64 reference sums.  FP64 storage: all zero.
int set_reference(elb_ctx *c, double n_r, double u_r, double T_r)
{
    int Q = c->Q, QP = padded_q(Q), N = c->N;
    std::vector<double> cref(QP, 0.0), gref(Q, 0.0);
    c->ref.assign(2 * Q, 0.0);
    for (int m = 0; m < 6; ++m) c->ref_sum[m] = 0.0;
    c->n_ref = n_r; c->u_ref = u_r; c->T_ref = T_r;
    if (c->P.precision != ELB_FP64) {
        std::vector<double> cc(QP, 0.0);
        cc[0] = 1.0;
        if (N >= 1) cc[1] = u_r;
        for (int l = 1; l < N; ++l)
            cc[l + 1] = (u_r * cc[l] + (T_r - 1.0) * std::sqrt((double)l) * cc[l - 1]) / std::sqrt((double)(l + 1));
        for (int l = 0; l <= N; ++l) cref[l] = n_r * cc[l];
        for (int k = 0; k < Q; ++k) {
            double g = 0.0;
            for (int l = 0; l <= N; ++l) g += c->Btd[(size_t)l * QP + k] * cref[l];
            gref[k] = g;
            c->ref[k] = g;
            c->ref[Q + k] = 2.0 * T_r * g;
        }
        for (int k = 0; k < Q; ++k) {
            double pk = c->p[k];
            c->ref_sum[0] += c->ref[k];
            c->ref_sum[1] += pk * c->ref[k];
            c->ref_sum[2] += pk * pk * c->ref[k];
            c->ref_sum[3] += pk * pk * pk * c->ref[k];
            c->ref_sum[4] += c->ref[Q + k];
            c->ref_sum[5] += pk * c->ref[Q + k];
        }
    }
    hipError_t e = hipMemcpyAsync(c->dev<double>(c->L.cref), cref.data(), sizeof(double) * QP, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->dev<double>(c->L.gref), gref.data(), sizeof(double) * Q, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->dev<double>(c->L.ref), c->ref.data(), sizeof(double) * 2 * Q, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_check(c, e, "reference upload");
}

// Fill all three levels (every row, ghosts included) with the equilibrium of the row
// fields held in the `rows` buffer.
int init_levels_from_rows(elb_ctx *c)
{
    int R = c->P.nx + 2 * NG, Q = c->Q, QP = padded_q(Q);
    int threads = 256, blocks = (R * Q + threads - 1) / threads;
    const double *rn = c->dev<double>(c->L.rows);
    const double *ru = rn + R, *rT = rn + 2 * R;
    bool book = c->P.precision == ELB_FP32_MIXED;
    for (int s = 0; s < 3; ++s) {
        double *U = book ? c->dev<double>(c->L.U[s]) : nullptr;
        if (c->P.precision == ELB_FP64)
            hipLaunchKernelGGL(k_init_equilibrium<double>, dim3(blocks), dim3(threads), 0, c->stream,
                               c->dev<double>(c->L.psi[s]), U, rn, ru, rT, c->dev<double>(c->L.btd),
                               c->dev<double>(c->L.sq), c->dev<double>(c->L.rsq),
                               c->dev<double>(c->L.ref), R, Q, QP, c->N);
        else
            hipLaunchKernelGGL(k_init_equilibrium<float>, dim3(blocks), dim3(threads), 0, c->stream,
                               c->dev<float>(c->L.psi[s]), U, rn, ru, rT, c->dev<double>(c->L.btd),
                               c->dev<double>(c->L.sq), c->dev<double>(c->L.rsq),
                               c->dev<double>(c->L.ref), R, Q, QP, c->N);
    }
    return hip_check(c, hipGetLastError(), "init kernel launch");
}

int run_moments(elb_ctx *c)
{
    int nx = c->P.nx, Q = c->Q;
    double *o = c->dev<double>(c->L.out);
    int threads = 256, blocks = (nx + threads - 1) / threads;
    const double *U = c->P.precision == ELB_FP32_MIXED ? c->dev<double>(c->L.U[0]) : nullptr;
    if (c->P.precision == ELB_FP64)
        hipLaunchKernelGGL(k_moments<double>, dim3(blocks), dim3(threads), 0, c->stream,
                           c->dev<double>(c->L.psi[0]), c->dev<double>(c->L.ref), U, c->dev<double>(c->L.p), nx, Q, o, o + nx,
                           o + 2 * nx, o + 3 * nx, o + 4 * nx, c->dev<double>(c->L.cons));
    else
        hipLaunchKernelGGL(k_moments<float>, dim3(blocks), dim3(threads), 0, c->stream,
                           c->dev<float>(c->L.psi[0]), c->dev<double>(c->L.ref), U, c->dev<double>(c->L.p), nx, Q, o, o + nx,
                           o + 2 * nx, o + 3 * nx, o + 4 * nx, c->dev<double>(c->L.cons));
    return hip_check(c, hipGetLastError(), "moments kernel launch");
}

int check_flag(elb_ctx *c)
{
    int flag = 0;
    int rc = hip_check(c, hipMemcpyAsync(&flag, c->dev<int>(c->L.flag), sizeof(int),
                                         hipMemcpyDeviceToHost, c->stream), "flag copy");
    if (rc) return rc;
    rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
    if (rc) return rc;
    if (flag) return fail(c, ELB_ENONFINITE, "a cell reached n <= 0, T <= 0 or non-finite moments");
    return ELB_OK;
}

}  // namespace

extern "C" {

int elb_supported_q(int32_t *out, int32_t cap)
{
    int n = (int)(sizeof kSupportedQ / sizeof kSupportedQ[0]);
    for (int i = 0; i < n && i < cap && out; ++i) out[i] = kSupportedQ[i];
    return n;
}

int elb_quadrature(int32_t q, double *nodes, double *weights)
{
    if (q < 1 || q > 256 || !nodes || !weights) return ELB_EINVAL;
    return gauss_hermite(q, nodes, weights) == 0 ? ELB_OK : ELB_EINVAL;
}

int elb_derived(const elb_params *p, double out[7])
{
    if (!out) return ELB_EINVAL;
    int N;
    double dx, dt, b, mu, eta0, chi0;
    std::string msg;
    int rc = derive(p, &N, &dx, &dt, &b, &mu, &eta0, &chi0, nullptr, &msg);
    if (rc) return rc;
    out[0] = dx; out[1] = dt; out[2] = b; out[3] = mu; out[4] = eta0; out[5] = chi0; out[6] = N;
    return ELB_OK;
}

int64_t elb_workspace_bytes(const elb_params *p)
{
    int N;
    double dx, dt, b, mu, eta0, chi0;
    std::string msg;
    if (derive(p, &N, &dx, &dt, &b, &mu, &eta0, &chi0, nullptr, &msg)) return -1;
    return (int64_t)make_layout(p->nx, p->q, N, p->precision).total;
}

int elb_create(const elb_params *p, void *dev_workspace, int64_t workspace_bytes, void *hip_stream,
               elb_ctx **out)
{
    if (!out) return ELB_EINVAL;
    *out = nullptr;
    elb_ctx *c = new (std::nothrow) elb_ctx();
    if (!c) return ELB_ENOMEM;
    std::string msg;
    int rc = derive(p, &c->N, &c->dx, &c->dt, &c->b, &c->mu_ref, &c->eta0, &c->chi0, &c->p, &msg);
    if (rc) { delete c; return rc; }
    c->P = *p;
    c->Q = p->q;
    c->L = make_layout(p->nx, p->q, c->N, p->precision);
    if (!dev_workspace || workspace_bytes < (int64_t)c->L.total) { delete c; return ELB_ENOMEM; }
    if (((uintptr_t)dev_workspace) & 255) { delete c; return ELB_EINVAL; }
    c->ws = (char *)dev_workspace;
    c->stream = (hipStream_t)hip_stream;
    int Q = c->Q, N = c->N;
    c->w.resize(Q);
    gauss_hermite(Q, c->p.data(), c->w.data());
    // Bt[l][k] = w_k h_l(p_k), h_l = He_l / sqrt(l!), zero-padded to QP x QP
    const int QP = padded_q(Q);
    c->Btd.assign((size_t)QP * QP, 0.0);
    std::vector<double> h(Q + 2);
    for (int k = 0; k < Q; ++k) {
        hermite_orthonormal(N, c->p[k], h.data());
        for (int l = 0; l <= N; ++l) c->Btd[(size_t)l * QP + k] = c->w[k] * h[l];
    }
    std::vector<float> btf(c->Btd.begin(), c->Btd.end());
    std::vector<double> sq(MAXQP + 2, 0.0), rsq(MAXQP + 2, 0.0);
    for (int l = 0; l < MAXQP + 2; ++l) {
        sq[l] = std::sqrt((double)l);
        rsq[l] = l ? 1.0 / std::sqrt((double)l) : 0.0;
    }
    hipError_t e = hipMemcpyAsync(c->dev<double>(c->L.p), c->p.data(), sizeof(double) * Q, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->dev<double>(c->L.btd), c->Btd.data(), sizeof(double) * c->Btd.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->dev<float>(c->L.btf), btf.data(), sizeof(float) * btf.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->dev<double>(c->L.sq), sq.data(), sizeof(double) * (QP + 2), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->dev<double>(c->L.rsq), rsq.data(), sizeof(double) * (QP + 2), hipMemcpyHostToDevice, c->stream);
    std::vector<double> rec(2 * QP, 0.0);
    for (int l = 0; l < QP; ++l) {
        rec[l] = l ? 1.0 / std::sqrt((double)l) : 0.0;
        rec[QP + l] = std::sqrt((double)l / (double)(l + 1));
    }
    if (e == hipSuccess) e = hipMemcpyAsync(c->dev<double>(c->L.rec), rec.data(), sizeof(double) * rec.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->dev<int>(c->L.flag), 0, sizeof(int) * 4, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { delete c; return ELB_EHIP; }
    if (set_reference(c, 1.0, 0.0, 1.0) != ELB_OK) { delete c; return ELB_EHIP; }
    *out = c;
    return ELB_OK;
}

int elb_set_state_moments(elb_ctx *c, const double *n, const double *u, const double *T)
{
    if (!c) return ELB_EINVAL;
    if (!n || !u || !T) return fail(c, ELB_EINVAL, "NULL input array");
    int nx = c->P.nx, R = nx + 2 * NG;
    std::vector<double> rows(3 * (size_t)R);
    double min_tau = 1e300;
    for (int i = 0; i < nx; ++i) {
        if (!(n[i] > 0) || !(T[i] > 0) || !std::isfinite(n[i]) || !std::isfinite(u[i]) || !std::isfinite(T[i]))
            return fail(c, ELB_EINVAL, "cell %d: need finite n > 0, T > 0", i);
        if (0.25 * c->b * n[i] >= 0.99) return fail(c, ELB_EINVAL, "cell %d: reduced density eta >= 0.99", i);
        min_tau = std::fmin(min_tau, host_tau(c, n[i], T[i]));
    }
    for (int r = 0; r < R; ++r) {
        int cell = r - NG;
        double vn, vu, vT;
        if (cell >= 0 && cell < nx) { vn = n[cell]; vu = u[cell]; vT = T[cell]; }
        else if (c->P.bc == ELB_BC_PERIODIC) {
            int w = ((cell % nx) + nx) % nx;
            vn = n[w]; vu = u[w]; vT = T[w];
        } else {
            const double *g = cell < 0 ? c->P.ghost_left : c->P.ghost_right;
            vn = g[0]; vu = g[1]; vT = g[2];
            min_tau = std::fmin(min_tau, host_tau(c, vn, vT));
        }
        rows[r] = vn; rows[R + r] = vu; rows[2 * R + r] = vT;
    }
    if (c->dt > 2.5 * min_tau)
        return fail(c, ELB_EINVAL, "dt = %g exceeds the RK3 stability limit 2.5 min tau = %g", c->dt, 2.5 * min_tau);
    {
        double sn = 0, su = 0, sT = 0;
        for (int i = 0; i < nx; ++i) { sn += n[i]; su += u[i]; sT += T[i]; }
        int rr = set_reference(c, sn / nx, su / nx, sT / nx);
        if (rr) return rr;
    }
    int rc = hip_check(c, hipMemcpyAsync(c->dev<double>(c->L.rows), rows.data(), sizeof(double) * rows.size(),
                                         hipMemcpyHostToDevice, c->stream), "rows copy");
    if (rc) return rc;
    rc = init_levels_from_rows(c);
    if (rc) return rc;
    rc = hip_check(c, hipMemsetAsync(c->dev<int>(c->L.flag), 0, sizeof(int) * 4, c->stream), "flag reset");
    if (rc) return rc;
    rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
    if (rc) return rc;
    c->has_state = true;
    c->steps = 0;
    return ELB_OK;
}

int elb_set_state_dist(elb_ctx *c, const double *phi, const double *theta)
{
    if (!c) return ELB_EINVAL;
    if (!phi || !theta) return fail(c, ELB_EINVAL, "NULL input array");
    if (!c->has_state && c->P.bc == ELB_BC_EQUILIBRIUM) {
        // ghost rows need the equilibrium of the end states: set them from a uniform state
        // first (interior rows are overwritten below)
        std::vector<double> n(c->P.nx, c->P.ghost_left[0]), u(c->P.nx, c->P.ghost_left[1]), T(c->P.nx, c->P.ghost_left[2]);
        int rc = elb_set_state_moments(c, n.data(), u.data(), T.data());
        if (rc) return rc;
    }
    int nx = c->P.nx, Q = c->Q, R = nx + 2 * NG;
    for (size_t j = 0; j < (size_t)nx * Q; ++j)
        if (!std::isfinite(phi[j]) || !std::isfinite(theta[j])) return fail(c, ELB_EINVAL, "non-finite distribution value");
    std::vector<double> old_ref = c->ref;
    if (c->P.precision != ELB_FP64) {
        // reference of the deviation storage: mean primitive state of the given cells
        double sn = 0, su = 0, sT = 0;
        for (int i = 0; i < nx; ++i) {
            double n = 0, j = 0, e = 0;
            for (int k = 0; k < Q; ++k) {
                double v = phi[(size_t)i * Q + k];
                n += v;
                j += c->p[k] * v;
                e += 0.5 * (c->p[k] * c->p[k] * v + theta[(size_t)i * Q + k]);
            }
            double u = j / n;
            sn += n; su += u; sT += (2.0 * e / n - u * u) / 3.0;
        }
        if (!(sn > 0) || !(sT > 0) || !std::isfinite(su)) return fail(c, ELB_EINVAL, "distributions with non-positive mean density or temperature");
        int rr = set_reference(c, sn / nx, su / nx, sT / nx);
        if (rr) return rr;
    }
    int es = elem_size(c->P.precision);
    std::vector<char> host((size_t)R * 2 * Q * es);
    // start from the current level 0 so ghost rows are preserved
    if (c->has_state) {
        int rc = hip_check(c, hipMemcpyAsync(host.data(), c->dev<char>(c->L.psi[0]), host.size(), hipMemcpyDeviceToHost, c->stream), "dist copy");
        if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
        if (rc) return rc;
    }
    // ghost rows (kept from the current state) move to the new reference
    if (es == 4 && c->has_state && old_ref.size() == (size_t)2 * Q) {
        for (int r = 0; r < R; ++r) {
            if (r >= NG && r < nx + NG) continue;
            for (int m = 0; m < 2 * Q; ++m) {
                float *v = (float *)host.data() + (size_t)r * 2 * Q + m;
                *v = (float)((double)*v + old_ref[m] - c->ref[m]);
            }
        }
    }
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < Q; ++k) {
            size_t o = (size_t)(i + NG) * 2 * Q + k;
            if (es == 8) {
                ((double *)host.data())[o] = phi[(size_t)i * Q + k];
                ((double *)host.data())[o + Q] = theta[(size_t)i * Q + k];
            } else {
                ((float *)host.data())[o] = (float)(phi[(size_t)i * Q + k] - c->ref[k]);
                ((float *)host.data())[o + Q] = (float)(theta[(size_t)i * Q + k] - c->ref[Q + k]);
            }
        }
    for (int s = 0; s < 3; ++s) {
        int rc = hip_check(c, hipMemcpyAsync(c->dev<char>(c->L.psi[s]), host.data(), host.size(), hipMemcpyHostToDevice, c->stream), "dist upload");
        if (rc) return rc;
        if (c->P.precision == ELB_FP32_MIXED) {
            // conserved densities of the stored (FP32) distributions, summed in FP64
            hipLaunchKernelGGL(k_conserved_from_psi<float>, dim3((R + 255) / 256), dim3(256), 0, c->stream,
                               c->dev<float>(c->L.psi[s]), c->dev<double>(c->L.ref),
                               c->dev<double>(c->L.U[s]), c->dev<double>(c->L.p), R, Q);
            rc = hip_check(c, hipGetLastError(), "conserved kernel launch");
            if (rc) return rc;
        }
    }
    int rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
    if (rc) return rc;
    c->has_state = true;
    c->steps = 0;
    return ELB_OK;
}

int elb_step(elb_ctx *c, int64_t nsteps)
{
    if (!c) return ELB_EINVAL;
    if (!c->has_state) return fail(c, ELB_ESTATE, "no state set");
    if (nsteps < 0) return fail(c, ELB_EINVAL, "nsteps < 0");
    for (int64_t s = 0; s < nsteps; ++s) {
        launch_stage(c, 0, 1, 0.0, 1.0, 1.0);                   // psi1 = psi + dt L[psi]
        launch_stage(c, 1, 2, 0.75, 0.25, 0.25);                // psi2 = 3/4 psi + 1/4 psi1 + 1/4 dt L[psi1]
        launch_stage(c, 2, 0, 1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0); // psi' = 1/3 psi + 2/3 psi2 + 2/3 dt L[psi2]
    }
    c->steps += nsteps;
    return hip_check(c, hipGetLastError(), "stage launch");
}

int elb_get_moments(elb_ctx *c, double *n, double *u, double *T, double *qx, double *pxx)
{
    if (!c) return ELB_EINVAL;
    if (!c->has_state) return fail(c, ELB_ESTATE, "no state set");
    int rc = run_moments(c);
    if (rc) return rc;
    int nx = c->P.nx;
    double *dst[5] = {n, u, T, qx, pxx};
    for (int f = 0; f < 5; ++f)
        if (dst[f]) {
            rc = hip_check(c, hipMemcpyAsync(dst[f], c->dev<double>(c->L.out) + (size_t)f * nx, sizeof(double) * nx,
                                             hipMemcpyDeviceToHost, c->stream), "moments copy");
            if (rc) return rc;
        }
    return check_flag(c);
}

int elb_get_dist(elb_ctx *c, double *phi, double *theta)
{
    if (!c) return ELB_EINVAL;
    if (!c->has_state) return fail(c, ELB_ESTATE, "no state set");
    int nx = c->P.nx, Q = c->Q, R = nx + 2 * NG, es = elem_size(c->P.precision);
    std::vector<char> host((size_t)R * 2 * Q * es);
    int rc = hip_check(c, hipMemcpyAsync(host.data(), c->dev<char>(c->L.psi[0]), host.size(), hipMemcpyDeviceToHost, c->stream), "dist copy");
    if (!rc) rc = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
    if (rc) return rc;
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < Q; ++k) {
            size_t o = (size_t)(i + NG) * 2 * Q + k;
            double vp = es == 8 ? ((double *)host.data())[o] : (double)((float *)host.data())[o] + c->ref[k];
            double vt = es == 8 ? ((double *)host.data())[o + Q] : (double)((float *)host.data())[o + Q] + c->ref[Q + k];
            if (phi) phi[(size_t)i * Q + k] = vp;
            if (theta) theta[(size_t)i * Q + k] = vt;
        }
    return check_flag(c);
}

int elb_get_conserved(elb_ctx *c, double out[3])
{
    if (!c || !out) return ELB_EINVAL;
    if (!c->has_state) return fail(c, ELB_ESTATE, "no state set");
    int rc = run_moments(c);
    if (rc) return rc;
    int nx = c->P.nx;
    std::vector<double> cons(3 * (size_t)nx);
    rc = hip_check(c, hipMemcpyAsync(cons.data(), c->dev<double>(c->L.cons), sizeof(double) * cons.size(),
                                     hipMemcpyDeviceToHost, c->stream), "conserved copy");
    if (rc) return rc;
    rc = check_flag(c);
    if (rc) return rc;
    double m = 0, j = 0, e = 0;
    for (int i = 0; i < nx; ++i) { m += cons[3 * i]; j += cons[3 * i + 1]; e += cons[3 * i + 2]; }
    out[0] = m * c->dx; out[1] = j * c->dx; out[2] = e * c->dx;
    return ELB_OK;
}

int elb_get_time(const elb_ctx *c, double *dt, int64_t *steps)
{
    if (!c) return ELB_EINVAL;
    if (dt) *dt = c->dt;
    if (steps) *steps = c->steps;
    return ELB_OK;
}

const char *elb_last_error(const elb_ctx *c)
{
    if (!c) return "NULL context";
    return c->err.c_str();
}

int elb_destroy(elb_ctx *c)
{
    if (!c) return ELB_EINVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    delete c;
    return e == hipSuccess ? ELB_OK : ELB_EHIP;
}

}  // extern "C"
