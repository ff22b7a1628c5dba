// hb_reduce.hip -- reductions and vector updates on the context's stream.
// Sums use a fixed number of blocks and fixed tree orders, so every run
// gives the same bits; max-norms are order independent.
#include "hb_internal.h"

namespace hb {

static constexpr int kT = 256;

__global__ void k_set(double* p, double v) { *p = v; }

void set_slot_zero(Ctx* c, int slot) { k_set<<<1, 1, 0, c->s>>>(c->sc + slot, 0.0); }
void set_slot(Ctx* c, int slot, double v) { k_set<<<1, 1, 0, c->s>>>(c->sc + slot, v); }

__global__ void k_maxabs(const double* __restrict__ v, long n, double* __restrict__ out)
{
    __shared__ unsigned long long sh[kT / 64];
    unsigned long long m = 0ull;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const unsigned long long b = abits(v[i]);
        m = b > m ? b : m;
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) atomic_max_bits(out, m);
}

void red_maxabs(Ctx* c, const double* v, long n, int slot, bool accumulate)
{
    if (!accumulate) set_slot_zero(c, slot);
    if (n <= 0) return;
    const long nb = (n + kT - 1) / kT;
    k_maxabs<<<(unsigned)(nb < kRedBlocks ? nb : kRedBlocks), kT, 0, c->s>>>(v, n, c->sc + slot);
}

// partial sums of v (or of a*b): block b owns the fixed index set
// {b*T + t + k*nblocks*T}
__global__ void k_sum_partial(const double* __restrict__ a, const double* __restrict__ b, long n, double* __restrict__ part)
{
    __shared__ double sh[kT / 64];
    double s = 0.0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        s += b ? a[i] * b[i] : a[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_sum_final(const double* __restrict__ part, int nb, double* __restrict__ out)
{
    __shared__ double sh[kT / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s;
}

static void sum_impl(Ctx* c, const double* a, const double* b, long n, int slot)
{
    k_sum_partial<<<kRedBlocks, kT, 0, c->s>>>(a, b, n, c->partial);
    k_sum_final<<<1, kT, 0, c->s>>>(c->partial, kRedBlocks, c->sc + slot);
}

void red_sum(Ctx* c, const double* v, long n, int slot) { sum_impl(c, v, nullptr, n, slot); }
void red_dot(Ctx* c, const double* a, const double* b, long n, int slot) { sum_impl(c, a, b, n, slot); }

void fetch_slots(Ctx* c)
{
    (void)hipMemcpyAsync(c->hsc, c->sc, sizeof(double) * S_NSLOT, hipMemcpyDeviceToHost, c->s);
    (void)hipStreamSynchronize(c->s);
}

// v -= sum(v) / n, the sum taken from the slot (no host round trip)
__global__ void k_sub_mean(double* __restrict__ v, long n, const double* __restrict__ sum)
{
    const double m = *sum / (double)n;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) v[i] -= m;
}

void sub_mean(Ctx* c, double* v, long n)
{
    red_sum(c, v, n, S_SUM);
    const long nb = (n + kT - 1) / kT;
    k_sub_mean<<<(unsigned)(nb < 4096 ? nb : 4096), kT, 0, c->s>>>(v, n, c->sc + S_SUM);
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

void copy(Ctx* c, double* dst, const double* src, long n)
{
    const long nb = (n + kT - 1) / kT;
    k_copy<<<(unsigned)(nb < 8192 ? nb : 8192), kT, 0, c->s>>>(dst, src, n);
}

__global__ void k_fill(double* __restrict__ d, double v, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = v;
}

void fill(Ctx* c, double* dst, double v, long n)
{
    const long nb = (n + kT - 1) / kT;
    k_fill<<<(unsigned)(nb < 8192 ? nb : 8192), kT, 0, c->s>>>(dst, v, n);
}

// ---- BiCGStab updates, with the scalars read from device slots ------------

__global__ void k_bicg_scalars(double* sc, int which)
{
    if (which == 0) {            // initial values
        sc[S_RHOP] = 1.0;
        sc[S_ALPHA] = 1.0;
        sc[S_OMEGA] = 1.0;
    } else if (which == 1) {     // rho and beta
        const double rho = sc[S_DOT0];
        sc[S_RHO] = rho;
        sc[S_BETA] = (rho / sc[S_RHOP]) * (sc[S_ALPHA] / sc[S_OMEGA]);
    } else if (which == 2) {     // alpha
        sc[S_ALPHA] = sc[S_RHO] / sc[S_DOT1];
    } else {                     // omega from (t.t, t.s); rho_prev = rho
        const double tt = sc[S_DOT0];
        sc[S_OMEGA] = tt > 0.0 ? sc[S_DOT1] / tt : 0.0;
        sc[S_RHOP] = sc[S_RHO];
    }
}

void bicg_init_scalars(Ctx* c) { k_bicg_scalars<<<1, 1, 0, c->s>>>(c->sc, 0); }
void bicg_beta(Ctx* c) { k_bicg_scalars<<<1, 1, 0, c->s>>>(c->sc, 1); }
void bicg_alpha(Ctx* c) { k_bicg_scalars<<<1, 1, 0, c->s>>>(c->sc, 2); }
void bicg_omega(Ctx* c) { k_bicg_scalars<<<1, 1, 0, c->s>>>(c->sc, 3); }

__global__ void k_bicg_p_dev(double* __restrict__ p, const double* __restrict__ r, const double* __restrict__ v,
                             const double* __restrict__ sc, long n)
{
    const double beta = sc[S_BETA], omega = sc[S_OMEGA];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

void bicg_p_dev(Ctx* c, double* p, const double* r, const double* v, long n)
{
    const long nb = (n + kT - 1) / kT;
    k_bicg_p_dev<<<(unsigned)(nb < 8192 ? nb : 8192), kT, 0, c->s>>>(p, r, v, c->sc, n);
}

__global__ void k_sub_scaled_max_dev(double* __restrict__ out, const double* __restrict__ a, const double* __restrict__ sp,
                                     const double* __restrict__ b, long n, double* __restrict__ mx)
{
    __shared__ unsigned long long sh[kT / 64];
    const double s = *sp;
    unsigned long long m = 0ull;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double v = a[i] - s * b[i];
        out[i] = v;
        const unsigned long long bb = abits(v);
        m = bb > m ? bb : m;
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) atomic_max_bits(mx, m);
}

void sub_scaled_max_dev(Ctx* c, double* out, const double* a, int sslot, const double* b, long n, int mslot)
{
    set_slot_zero(c, mslot);
    const long nb = (n + kT - 1) / kT;
    k_sub_scaled_max_dev<<<(unsigned)(nb < kRedBlocks ? nb : kRedBlocks), kT, 0, c->s>>>(out, a, c->sc + sslot, b, n,
                                                                                           c->sc + mslot);
}

// x += alpha ph + omega sh (with_omega), or x = alpha ph + x
__global__ void k_bicg_x_dev(double* __restrict__ x, const double* __restrict__ ph, const double* __restrict__ sh_,
                             const double* __restrict__ sc, int with_omega, long n)
{
    const double alpha = sc[S_ALPHA], omega = sc[S_OMEGA];
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        if (with_omega) x[i] += alpha * ph[i] + omega * sh_[i];
        else x[i] = alpha * ph[i] + 1.0 * x[i];
    }
}

void bicg_x_dev(Ctx* c, double* x, const double* ph, const double* sh, bool with_omega, long n)
{
    const long nb = (n + kT - 1) / kT;
    k_bicg_x_dev<<<(unsigned)(nb < 8192 ? nb : 8192), kT, 0, c->s>>>(x, ph, sh, c->sc, with_omega ? 1 : 0, n);
}

// ---- precision conversions of the mixed-precision correction cycles ---------

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, float* __restrict__ zero, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        dst[i] = (float)src[i];
        if (zero) zero[i] = 0.0f;
    }
}

void to_f32(Ctx* c, const double* src, float* dst, float* zero, long n)
{
    const long nb = (n + kT - 1) / kT;
    k_to_f32<<<(unsigned)(nb < 8192 ? nb : 8192), kT, 0, c->s>>>(src, dst, zero, n);
}

__global__ void k_add_f32(double* __restrict__ x, const float* __restrict__ e, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] += (double)e[i];
}

void add_f32(Ctx* c, double* x, const float* e, long n)
{
    const long nb = (n + kT - 1) / kT;
    k_add_f32<<<(unsigned)(nb < 8192 ? nb : 8192), kT, 0, c->s>>>(x, e, n);
}

__global__ void k_from_f32(const float* __restrict__ e, double* __restrict__ x, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = (double)e[i];
}

void from_f32(Ctx* c, const float* e, double* x, long n)
{
    const long nb = (n + kT - 1) / kT;
    k_from_f32<<<(unsigned)(nb < 8192 ? nb : 8192), kT, 0, c->s>>>(e, x, n);
}

}  // namespace hb
