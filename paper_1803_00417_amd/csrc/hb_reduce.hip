// hb_reduce.hip -- reductions and vector updates on the context's stream,
// single-array and segmented over a batch of cavities (block y = cavity).
// Sums use a fixed number of blocks per cavity and fixed tree orders, so
// every run gives the same bits, and a cavity's sum does not depend on the
// other cavities of the batch; max-norms are order independent.
#include "hb_internal.h"

#include <chrono>

namespace hb {

static constexpr int kT = 256;

// Blocks per cavity of a max-norm whose blocks meet on one slot: every
// block's atomic queues on that address, so a few long blocks beat many
// short ones while they still stream the vector at full rate (a maximum is
// exact in any order): one block per 8192 values, between 64 and
// kRedBlocks.
static long maxnorm_blocks(long n)
{
    const long b = n / 8192;
    return b < 64 ? 64 : (b > kRedBlocks ? kRedBlocks : b);
}

static unsigned blocks_for(long n, long cap)
{
    const long nb = (n + kT - 1) / kT;
    return (unsigned)(nb < 1 ? 1 : (nb < cap ? nb : cap));
}

// ---- single arrays ----------------------------------------------------------

__global__ void k_set(double* p, double v) { *p = v; }

void set_slot(Ctx* c, int cav, int slot, double v) { k_set<<<1, 1, 0, c->s>>>(c->sc + (long)cav * S_NSLOT + slot, v); }

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

void red_maxabs(Ctx* c, int cav, const double* v, long n, int slot)
{
    double* out = c->sc + (long)cav * S_NSLOT + slot;
    k_set<<<1, 1, 0, c->s>>>(out, 0.0);
    if (n <= 0) return;
    k_maxabs<<<blocks_for(n, maxnorm_blocks(n)), kT, 0, c->s>>>(v, n, out);
}

// largest |a - b| (the change of a field over a step)
__global__ void k_maxdiff(const double* __restrict__ a, const double* __restrict__ b, long n, double* __restrict__ out)
{
    __shared__ unsigned long long sh[kT / 64];
    unsigned long long m = 0ull;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const unsigned long long d = abits(a[i] - b[i]);
        m = d > m ? d : m;
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) atomic_max_bits(out, m);
}

void red_maxdiff(Ctx* c, int cav, const double* a, const double* b, long n, int slot)
{
    double* out = c->sc + (long)cav * S_NSLOT + slot;
    k_set<<<1, 1, 0, c->s>>>(out, 0.0);
    if (n <= 0) return;
    k_maxdiff<<<blocks_for(n, maxnorm_blocks(n)), kT, 0, c->s>>>(a, b, n, out);
}

// Publication of the slots: one block copies them into the coherent pinned
// mirror, every thread makes its writes visible system-wide, then one
// release store sets the publication word.  The host spins on that word: it
// is set once every earlier command of the stream has completed (in-order
// stream), which is all a synchronisation would give, without the copy
// command and the wake-up of a blocking wait.
__global__ void k_publish(const double* __restrict__ sc, double* hsc, int n, unsigned long long* seq,
                          unsigned long long want)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) hsc[i] = sc[i];
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(seq, want, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void fetch_slots(Ctx* c)
{
    flush_max_final(c);
    const int n = S_NSLOT * c->nb;
    const unsigned long long want = ++c->pub;
    k_publish<<<1, kT, 0, c->s>>>(c->sc, c->dhsc, n, c->dhseq, want);
    // spin for a bounded time, then block on the stream (a long segment of
    // work); if the word is still not visible, copy the slots the slow way
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned it = 1;; ++it) {
        if (__atomic_load_n(c->hseq, __ATOMIC_ACQUIRE) == want) {
            c->wait_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            ++c->waits;
            return;
        }
        __builtin_ia32_pause();
        if ((it & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) break;
    }
    (void)hipStreamSynchronize(c->s);
    if (__atomic_load_n(c->hseq, __ATOMIC_ACQUIRE) == want) return;
    (void)hipMemcpy(c->hsc, c->sc, sizeof(double) * n, hipMemcpyDeviceToHost);
}

// ---- convergence decisions on the device -----------------------------------

// The largest of a cavity's kSubMax partial words, read by one 256-thread
// block, and the words cleared: every load is issued before the first
// clear, so the pass costs one memory round trip rather than one per word.
__device__ inline unsigned long long take_max_words(unsigned long long* __restrict__ w)
{
    static_assert(kSubMax % 256 == 0, "whole words per thread");
    constexpr int PER = kSubMax / 256;
    unsigned long long v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] = w[threadIdx.x + 256 * u];
    unsigned long long m = 0ull;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        m = v[u] > m ? v[u] : m;
        w[threadIdx.x + 256 * u] = 0ull;
    }
    return m;
}

__device__ inline bool conv_stops(double* R, const ConvArgs& a)
{
    const double cyc = R[R_CYC];
    if (a.fixed) return cyc >= (double)a.max_cycles;
    if (R[R_REL] <= a.tol) return true;
    if (cyc >= (double)a.max_cycles) {
        R[R_RC] = (double)HB_ERR_NOCONV;
        return true;
    }
    return false;
}

// relative residual from slot S_MAX; false (and NONFINITE) when not finite
__device__ inline bool conv_take_rel(double* S, double* R)
{
    const double rel = S[S_MAX] / R[R_BN];
    R[R_REL] = rel;
    if (!isfinite(rel)) {
        R[R_RC] = (double)HB_ERR_NONFINITE;
        return false;
    }
    return true;
}

// One thread per cavity applies the check point's rule (the rules of a
// host-driven loop, in the same order), then the block counts the cavities
// still active and thread 0 publishes the count with the check point number
// by one system-scope release store into the pinned ring.
__global__ void __launch_bounds__(1024) k_conv(ConvArgs a, double* __restrict__ sc, int* __restrict__ act,
                                               int* __restrict__ act2, int* __restrict__ sel,
                                               unsigned long long* ring, unsigned long long* __restrict__ mp)
{
    __shared__ double sh[1024 / 64];
    __shared__ unsigned long long shm[1024 / 64];
    if (a.mf_slot >= 0) {
        // the max-norm's final pass (one cavity): the largest partial word,
        // the words cleared, the slot written when the cavity is active
        unsigned long long m = take_max_words(mp);
        m = block_umax(m, shm);
        if (threadIdx.x == 0 && (!a.mf_act || act[0])) sc[a.mf_slot] = __longlong_as_double((long long)m);
        __syncthreads();
    }
    double nact = 0.0;
    for (int i = threadIdx.x; i < a.nb; i += blockDim.x) {
        double* S = sc + (long)i * S_NSLOT;
        double* R = S + a.rec;
        switch (a.mode) {
        case CV_BEGIN: {
            const double bn = S[S_MAX];
            const bool ok = isfinite(bn) && isfinite(S[S_MAX2]);
            R[R_BN] = bn;
            R[R_REL] = 0.0;
            R[R_CYC] = 0.0;
            R[R_RC] = ok ? (double)HB_OK : (double)HB_ERR_NONFINITE;
            act[i] = ok && bn != 0.0;
            act2[i] = ok && bn == 0.0;
            sel[i] = 0;
            break;
        }
        case CV_INIT:
        case CV_CYCLE:
            if (!act[i]) break;
            if (a.mode == CV_CYCLE) R[R_CYC] += 1.0;
            if (!conv_take_rel(S, R) || conv_stops(R, a)) {
                act[i] = 0;
                sel[i] = a.cur_sel;
            }
            break;
        case CV_HALF: {
            act2[i] = 0;
            if (!act[i]) break;
            R[R_CYC] += 1.0;
            if (S[S_RHO] == 0.0) {
                R[R_RC] = (double)HB_ERR_NOCONV;
                act[i] = 0;
                break;
            }
            const double srel = S[S_MAX] / R[R_BN];
            if ((!a.fixed && srel <= a.tol) || (a.fixed && R[R_CYC] >= (double)a.max_cycles)) {
                act2[i] = 1;
                act[i] = 0;
                R[R_REL] = srel;
            }
            break;
        }
        case CV_FULL:
            if (!act[i]) break;
            R[R_CYC] += 1.0;
            if (!conv_take_rel(S, R)) {
                act[i] = 0;
                break;
            }
            if (S[S_OMEGA] == 0.0) {
                R[R_RC] = (double)HB_ERR_NOCONV;
                act[i] = 0;
                break;
            }
            if (conv_stops(R, a)) act[i] = 0;
            break;
        case CV_END_PLAIN:
            act2[i] = R[R_BN] != 0.0 && R[R_RC] != (double)HB_ERR_NONFINITE;
            break;
        case CV_END_KRYLOV:
            act[i] = R[R_BN] != 0.0 && R[R_RC] != (double)HB_ERR_NONFINITE;
            break;
        case CV_FINAL:
            if (act[i]) conv_take_rel(S, R);
            break;
        }
        nact += act[i] != 0 ? 1.0 : 0.0;
    }
    nact = block_sum(nact, sh);
    if (threadIdx.x == 0 && a.seq) {
        // the host reads only this word (the count), so the store needs no
        // release ordering of the kernel's other writes: a relaxed
        // system-scope store reaches the coherent pinned ring without the
        // cache write-back a release would take
        const unsigned long long w = ((unsigned long long)nact << 32) | (a.seq & 0xffffffffull);
        __hip_atomic_store(ring + a.seq % kRing, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

void launch_conv(Ctx* c, ConvArgs a)
{
    a.mf_slot = -1;
    a.mf_act = 0;
    if (c->mf_slot >= 0) {
        // only the check's own act flags are read by the fused final pass
        if (c->mf_act && c->mf_act != c->act) {
            flush_max_final(c);
        } else {
            a.mf_slot = c->mf_slot;
            a.mf_act = c->mf_act != nullptr;
            c->mf_slot = -1;
        }
    }
    c->defer_mf = false;
    int nt = c->nb >= 1024 ? 1024 : ((c->nb + 63) / 64) * 64;
    if (a.mf_slot >= 0) nt = 256;
    k_conv<<<1, nt, 0, c->s>>>(a, c->sc, c->act, c->act2, c->sel, c->dring, c->mpart);
}

int wait_active(Ctx* c, unsigned long long seq)
{
    volatile unsigned long long* e = c->hring + seq % kRing;
    const unsigned long long lo = seq & 0xffffffffull;
    const auto t0 = std::chrono::steady_clock::now();
    for (unsigned it = 1;; ++it) {
        const unsigned long long w = __atomic_load_n(const_cast<unsigned long long*>(e), __ATOMIC_ACQUIRE);
        if ((w & 0xffffffffull) == lo) {
            c->wait_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            ++c->waits;
            return (int)(w >> 32);
        }
        __builtin_ia32_pause();
        if ((it & 1023) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) break;
    }
    (void)hipStreamSynchronize(c->s);
    const unsigned long long w = __atomic_load_n(const_cast<unsigned long long*>(e), __ATOMIC_ACQUIRE);
    return (w & 0xffffffffull) == lo ? (int)(w >> 32) : -1;
}

// per-cavity flags passed by value (a copy command costs the runtime more
// than a launch)
__global__ void k_set_flags(int* __restrict__ dev, FlagArgs a)
{
    const int i = threadIdx.x;
    if (i < a.n) dev[i] = a.v[i];
}

void set_flags(Ctx* c, int* dev, const int* host)
{
    if (c->nb <= kFlagArgs) {
        FlagArgs a;
        a.n = c->nb;
        for (int i = 0; i < c->nb; ++i) a.v[i] = host[i];
        k_set_flags<<<1, kFlagArgs, 0, c->s>>>(dev, a);
    } else {
        (void)hipMemcpyAsync(dev, host, sizeof(int) * c->nb, hipMemcpyHostToDevice, c->s);
    }
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

void copy(Ctx* c, double* dst, const double* src, long n)
{
    if (n > 0) k_copy<<<blocks_for(n, 8192), kT, 0, c->s>>>(dst, src, n);
}

__global__ void k_fill(double* __restrict__ d, double v, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = v;
}

void fill(Ctx* c, double* dst, double v, long n)
{
    if (n > 0) k_fill<<<blocks_for(n, 8192), kT, 0, c->s>>>(dst, v, n);
}

// slot of every active cavity = max of its partial words; the words of
// every cavity are cleared (a single-cavity launch writes them whether or
// not the cavity is flagged active)
__global__ void k_max_final(const int* __restrict__ act, unsigned long long* __restrict__ mp, double* __restrict__ sc,
                            int slot)
{
    __shared__ unsigned long long sh[kT / 64];
    const int cav = blockIdx.x;
    unsigned long long* w = mp + (long)cav * kSubMax;
    static_assert(kT == 256, "one 256-thread block per cavity");
    unsigned long long m = take_max_words(w);
    m = block_umax(m, sh);
    if (threadIdx.x == 0 && (!act || act[cav])) sc[(long)cav * S_NSLOT + slot] = __longlong_as_double((long long)m);
}

void launch_max_final(Ctx* c, const int* act, int slot)
{
    flush_max_final(c);
    if (c->defer_mf && c->nb == 1) {
        // the next convergence check does this pass (one launch fewer)
        c->defer_mf = false;
        c->mf_slot = slot;
        c->mf_act = act;
        return;
    }
    k_max_final<<<c->nb, kT, 0, c->s>>>(act, c->mpart, c->sc, slot);
}

void flush_max_final(Ctx* c)
{
    if (c->mf_slot < 0) return;
    const int slot = c->mf_slot;
    c->mf_slot = -1;
    k_max_final<<<c->nb, kT, 0, c->s>>>(c->mf_act, c->mpart, c->sc, slot);
}

// ---- stage fields of every cavity (tables c->ck, c->cio) ----------------------

// a stage field of one cavity and its length
__device__ inline const double* stage_field(const CavK& K, const CavIO& IO, int f, long& n)
{
    const long nv = (long)K.g.dim * K.nc;
    switch (f) {
    case SF_U: n = nv; return IO.u;
    case SF_P: n = K.nn; return IO.p;
    case SF_UOUT: n = nv; return IO.uout;
    case SF_RNODE: n = K.nn; return K.rnode;
    case SF_MACRHS: n = K.nc; return K.macrhs;
    case SF_USTAR: n = nv; return K.ustar;
    default: n = K.nn; return K.phi;
    }
}

// dst <- src of every cavity (block y = cavity)
__global__ void k_stage_copy(const CavK* __restrict__ ck, const CavIO* __restrict__ io, int dst, int src)
{
    const CavK& K = ck[blockIdx.y];
    const CavIO& IO = io[blockIdx.y];
    long n, m;
    double* d = const_cast<double*>(stage_field(K, IO, dst, n));
    const double* s = stage_field(K, IO, src, m);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

static long stage_longest(const Ctx* c)
{
    long mx = 1;
    for (const Cav& v : c->cv) mx = std::max(mx, std::max((long)v.dim * v.nc, v.nn));
    return mx;
}

void stage_copy(Ctx* c, int dst, int src)
{
    k_stage_copy<<<dim3(blocks_for(stage_longest(c), 8192), c->nb), kT, 0, c->s>>>(c->ck, c->cio, dst, src);
}

// max |field| of every cavity into its slot (the slot zeroed first); the
// same fixed block count per cavity as the single-array reduction
__global__ void k_stage_maxabs(const CavK* __restrict__ ck, const CavIO* __restrict__ io, int f, int slot)
{
    __shared__ unsigned long long sh[kT / 64];
    const CavK& K = ck[blockIdx.y];
    long n;
    const double* v = stage_field(K, io[blockIdx.y], f, n);
    unsigned long long m = 0ull;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const unsigned long long b = abits(v[i]);
        m = b > m ? b : m;
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) atomic_max_bits(K.sc + slot, m);
}

void stage_maxabs(Ctx* c, int field, int slot)
{
    seg_set_zero(c, slot);
    const long n = stage_longest(c);
    k_stage_maxabs<<<dim3(blocks_for(n, maxnorm_blocks(n)), c->nb), kT, 0, c->s>>>(c->ck, c->cio, field, slot);
}

// ---- segmented over the batch -------------------------------------------------

// this block's cavity segment; the block returns when the cavity is inactive
#define SEG_ENTER(sv, off, n)                                  \
    const int cav_ = blockIdx.y;                               \
    const long off = (sv).off[cav_], n = (sv).n[cav_];         \
    if ((sv).act && !(sv).act[cav_]) return;

#define SEG_LOOP(i, n) for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

static long seg_longest(const MG& m)
{
    long mx = 0;
    for (long v : m.L[0].hnu) mx = v > mx ? v : mx;
    return mx;
}

// the longest segment of any level-0 arena
static long seg_max_len(const Ctx* c)
{
    long mx = seg_longest(c->visc);
    const long a = seg_longest(c->mac), b = seg_longest(c->nodal);
    if (a > mx) mx = a;
    if (b > mx) mx = b;
    return mx;
}

// grid of a segmented launch: blocks per cavity sized for the longest
// segment of any level-0 arena, at most cap blocks in total
static dim3 seg_grid(const Ctx* c, long cap)
{
    const long mx = seg_max_len(c);
    long per = cap / c->nb;
    if (per < 1) per = 1;
    return dim3(blocks_for(mx, per), c->nb);
}

__global__ void k_seg_set(double* sc, int slot, int nb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) sc[(long)i * S_NSLOT + slot] = 0.0;
}

void seg_set_zero(Ctx* c, int slot) { k_seg_set<<<(c->nb + 63) / 64, 64, 0, c->s>>>(c->sc, slot, c->nb); }

__global__ void k_seg_maxabs(SegV sv, const double* __restrict__ v, double* __restrict__ sc, int slot)
{
    __shared__ unsigned long long sh[kT / 64];
    SEG_ENTER(sv, off, n);
    unsigned long long m = 0ull;
    SEG_LOOP(i, n)
    {
        const unsigned long long b = abits(v[off + i]);
        m = b > m ? b : m;
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) atomic_max_bits(sc + (long)cav_ * S_NSLOT + slot, m);
}

void seg_maxabs(Ctx* c, const SegV& s, const double* v, int slot)
{
    seg_set_zero(c, slot);
    k_seg_maxabs<<<seg_grid(c, maxnorm_blocks(seg_max_len(c)) * c->nb), kT, 0, c->s>>>(s, v, c->sc, slot);
}

__global__ void k_seg_set2(double* sc, int slot0, int slot1, int nb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) {
        sc[(long)i * S_NSLOT + slot0] = 0.0;
        sc[(long)i * S_NSLOT + slot1] = 0.0;
    }
}

// max |a| into slot0 and max |b| into slot1 of every cavity in one pass
__global__ void k_seg_maxabs2(SegV sv, const double* __restrict__ a, const double* __restrict__ b,
                              double* __restrict__ sc, int slot0, int slot1)
{
    __shared__ unsigned long long sh[kT / 64];
    SEG_ENTER(sv, off, n);
    unsigned long long ma = 0ull, mb = 0ull;
    SEG_LOOP(i, n)
    {
        const unsigned long long x = abits(a[off + i]), y = abits(b[off + i]);
        ma = x > ma ? x : ma;
        mb = y > mb ? y : mb;
    }
    ma = block_umax(ma, sh);
    mb = block_umax(mb, sh);
    if (threadIdx.x == 0) {
        atomic_max_bits(sc + (long)cav_ * S_NSLOT + slot0, ma);
        atomic_max_bits(sc + (long)cav_ * S_NSLOT + slot1, mb);
    }
}

void seg_maxabs2(Ctx* c, const SegV& s, const double* a, int slot0, const double* b, int slot1)
{
    k_seg_set2<<<(c->nb + 63) / 64, 64, 0, c->s>>>(c->sc, slot0, slot1, c->nb);
    k_seg_maxabs2<<<seg_grid(c, maxnorm_blocks(seg_max_len(c)) * c->nb), kT, 0, c->s>>>(s, a, b, c->sc, slot0,
                                                                                       slot1);
}

// BiCGStab's scalars, each in one place: the initial values, beta from the
// new rho, alpha from r^.v, omega from (t.t, t.s)
__device__ inline void bicg_init(double* sc)
{
    sc[S_RHOP] = 1.0;
    sc[S_ALPHA] = 1.0;
    sc[S_OMEGA] = 1.0;
}
__device__ inline double bicg_beta(const double* sc, double rho)
{
    return (rho / sc[S_RHOP]) * (sc[S_ALPHA] / sc[S_OMEGA]);
}
__device__ inline double bicg_alpha(const double* sc, double rv) { return sc[S_RHO] / rv; }
__device__ inline double bicg_omega(double tt, double ts) { return tt > 0.0 ? ts / tt : 0.0; }

// Dot products: a partial pass (one or two products of a with b0, b1 per
// block; block x of cavity y owns the index set {x*T + t + k*kRedBlocks*T},
// so every run gives the same bits) and a total of the partials in a fixed
// order, taken either by a final pass of one block per cavity (dot_total in
// k_seg_dot_final) or by every block of the kernel that uses the product
// (the BiCGStab updates below).  No block waits on another: a device-scope
// release per block would write back the XCD's L2 each time.  The partial
// pass also clears slot `zero` (-1: none), the max-norm slot the kernel
// after it fills with atomic maxima.
__global__ void k_seg_dot_partial(SegV sv, const double* __restrict__ a, const double* __restrict__ b0,
                                  const double* __restrict__ b1, double* __restrict__ part, double* __restrict__ scb,
                                  int zero)
{
    __shared__ double sh[kT / 64];
    SEG_ENTER(sv, off, n);
    if (zero >= 0 && blockIdx.x == 0 && threadIdx.x == 0) scb[(long)cav_ * S_NSLOT + zero] = 0.0;
    double s0 = 0.0, s1 = 0.0;
    SEG_LOOP(i, n)
    {
        s0 += b0 ? a[off + i] * b0[off + i] : a[off + i];
        if (b1) s1 += a[off + i] * b1[off + i];
    }
    s0 = block_sum(s0, sh);
    if (threadIdx.x == 0) part[(long)cav_ * kRedBlocks + blockIdx.x] = s0;
    if (b1) {
        s1 = block_sum(s1, sh);
        if (threadIdx.x == 0) part[((long)gridDim.y + cav_) * kRedBlocks + blockIdx.x] = s1;
    }
}

// total of partial row `row` (kRedBlocks words) in a block of kT threads:
// thread t adds words t, t + kT, ..., then the block's fixed tree; the
// result is returned to every thread
__device__ inline double dot_total(const double* __restrict__ part, long row, double* sh, double* bcast)
{
    double t0 = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) t0 += part[row * kRedBlocks + i];
    t0 = block_sum(t0, sh);
    if (threadIdx.x == 0) *bcast = t0;
    __syncthreads();
    return *bcast;
}

__global__ void k_seg_dot_final(SegV sv, const double* __restrict__ part, double* __restrict__ scb, int slot0,
                                int slot1)
{
    __shared__ double sh[kT / 64], bc;
    const int cav = blockIdx.x;
    if (sv.act && !sv.act[cav]) return;
    const double t0 = dot_total(part, cav, sh, &bc);
    const double t1 = slot1 >= 0 ? dot_total(part, (long)gridDim.x + cav, sh, &bc) : 0.0;
    if (threadIdx.x == 0) {
        double* sc = scb + (long)cav * S_NSLOT;
        sc[slot0] = t0;
        if (slot1 >= 0) sc[slot1] = t1;
    }
}

void seg_dot_part(Ctx* c, const SegV& s, const double* a, const double* b0, const double* b1, double* part, int zero)
{
    k_seg_dot_partial<<<dim3(kRedBlocks, c->nb), kT, 0, c->s>>>(s, a, b0, b1, part, c->sc, zero);
}

static void dot_launch(Ctx* c, const SegV& s, const double* a, const double* b0, const double* b1, int slot0, int slot1)
{
    seg_dot_part(c, s, a, b0, b1, c->partial, -1);
    k_seg_dot_final<<<c->nb, kT, 0, c->s>>>(s, c->partial, c->sc, slot0, b1 ? slot1 : -1);
}

void seg_dot(Ctx* c, const SegV& s, const double* a, const double* b, int slot)
{
    dot_launch(c, s, a, b, nullptr, slot, -1);
}

double* rho_partials(Ctx* c) { return c->partial + 2L * kRedBlocks * c->nb; }

// v -= sum(v) / n per cavity, every block totalling the sum's partials
// itself (block 0 records the sum in slot S_SUM)
__global__ void k_seg_sub_mean(SegV sv, double* __restrict__ v, double* __restrict__ sc,
                               const double* __restrict__ part)
{
    __shared__ double sh[kT / 64], bc;
    SEG_ENTER(sv, off, n);
    const double sum = dot_total(part, cav_, sh, &bc);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[(long)cav_ * S_NSLOT + S_SUM] = sum;
    const double m = sum / (double)n;
    SEG_LOOP(i, n) v[off + i] -= m;
}

void seg_sub_mean(Ctx* c, const SegV& s, double* v)
{
    seg_dot_part(c, s, v, nullptr, nullptr, c->partial, -1);
    k_seg_sub_mean<<<seg_grid(c, (long)kRedBlocks * c->nb), kT, 0, c->s>>>(s, v, c->sc, c->partial);
}

__global__ void k_seg_copy(SegV sv, double* __restrict__ d, const double* __restrict__ s)
{
    SEG_ENTER(sv, off, n);
    SEG_LOOP(i, n) d[off + i] = s[off + i];
}

void seg_copy(Ctx* c, const SegV& s, double* dst, const double* src)
{
    k_seg_copy<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, dst, src);
}

__global__ void k_seg_fill(SegV sv, double* __restrict__ d, double v)
{
    SEG_ENTER(sv, off, n);
    SEG_LOOP(i, n) d[off + i] = v;
}

void seg_fill(Ctx* c, const SegV& s, double* dst, double v)
{
    k_seg_fill<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, dst, v);
}

// dst = (sel[cavity] ? src1 : src0) over each cavity's segment
__global__ void k_seg_copy_sel(SegV sv, double* __restrict__ d, const double* __restrict__ s0,
                               const double* __restrict__ s1, const int* __restrict__ sel)
{
    SEG_ENTER(sv, off, n);
    const double* s = sel[cav_] ? s1 : s0;
    SEG_LOOP(i, n) d[off + i] = s[off + i];
}

void seg_copy_sel(Ctx* c, const SegV& s, double* dst, const double* src0, const double* src1, const int* sel)
{
    k_seg_copy_sel<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, dst, src0, src1, sel);
}

// ---- precision conversions of the mixed-precision correction cycles ---------

__global__ void k_seg_to_f32(SegV sv, const double* __restrict__ src, float* __restrict__ dst, float* __restrict__ zero)
{
    SEG_ENTER(sv, off, n);
    SEG_LOOP(i, n)
    {
        dst[off + i] = (float)src[off + i];
        if (zero) zero[off + i] = 0.0f;
    }
}

void seg_to_f32(Ctx* c, const SegV& s, const double* src, float* dst, float* zero)
{
    k_seg_to_f32<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, src, dst, zero);
}

__global__ void k_seg_add_f32(SegV sv, double* __restrict__ x, const float* __restrict__ e)
{
    SEG_ENTER(sv, off, n);
    SEG_LOOP(i, n) x[off + i] += (double)e[off + i];
}

void seg_add_f32(Ctx* c, const SegV& s, double* x, const float* e)
{
    k_seg_add_f32<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, x, e);
}

__global__ void k_seg_from_f32(SegV sv, const float* __restrict__ e, double* __restrict__ x)
{
    SEG_ENTER(sv, off, n);
    SEG_LOOP(i, n) x[off + i] = (double)e[off + i];
}

void seg_from_f32(Ctx* c, const SegV& s, const float* e, double* x)
{
    k_seg_from_f32<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, e, x);
}

__global__ void k_flat_to_f32(const double* __restrict__ src, float* __restrict__ dst, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

void flat_to_f32(Ctx* c, const double* src, float* dst, long n)
{
    if (n > 0) k_flat_to_f32<<<blocks_for(n, 8192), kT, 0, c->s>>>(src, dst, n);
}

// ---- BiCGStab updates, with each cavity's scalars read from its slots -------

__global__ void k_bicg_init(double* scb, int nb, const int* act)
{
    const int cav = blockIdx.x * blockDim.x + threadIdx.x;
    if (cav >= nb || (act && !act[cav])) return;
    bicg_init(scb + (long)cav * S_NSLOT);
}

void bicg_init_scalars(Ctx* c, const int* act)
{
    k_bicg_init<<<(c->nb + 63) / 64, 64, 0, c->s>>>(c->sc, c->nb, act);
}

// rho = r^.r from its partials (every block takes the same total), beta;
// p = r + beta (p - omega v).  Block 0 of the cavity records rho and beta.
__global__ void k_bicg_p_rho(SegV sv, double* __restrict__ p, const double* __restrict__ r,
                             const double* __restrict__ v, double* __restrict__ scb, const double* __restrict__ part)
{
    __shared__ double sh[kT / 64], bc;
    SEG_ENTER(sv, off, n);
    double* sc = scb + (long)cav_ * S_NSLOT;
    const double rho = dot_total(part, cav_, sh, &bc);
    const double beta = bicg_beta(sc, rho), omega = sc[S_OMEGA];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_DOT0] = rho;
        sc[S_RHO] = rho;
        sc[S_BETA] = beta;
    }
    SEG_LOOP(i, n) p[off + i] = r[off + i] + beta * (p[off + i] - omega * v[off + i]);
}

void bicg_p_rho(Ctx* c, const SegV& s, double* p, const double* r, const double* v, const double* part)
{
    k_bicg_p_rho<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, p, r, v, c->sc, part);
}

// alpha = rho / r^.v from its partials; s = r - alpha v, with the max-norm
// of s into slot mslot (cleared by the partial pass), or into the partial
// words mp.  Block 0 records r^.v and alpha.
__global__ void k_bicg_s_alpha(SegV sv, double* __restrict__ out, const double* __restrict__ r,
                               const double* __restrict__ v, double* __restrict__ scb, const double* __restrict__ part,
                               int mslot, unsigned long long* __restrict__ mp)
{
    __shared__ double shd[kT / 64], bc;
    __shared__ unsigned long long sh[kT / 64];
    SEG_ENTER(sv, off, n);
    double* sc = scb + (long)cav_ * S_NSLOT;
    const double rv = dot_total(part, cav_, shd, &bc);
    const double alpha = bicg_alpha(sc, rv);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_DOT1] = rv;
        sc[S_ALPHA] = alpha;
    }
    unsigned long long m = 0ull;
    SEG_LOOP(i, n)
    {
        const double w = r[off + i] - alpha * v[off + i];
        out[off + i] = w;
        const unsigned long long bb = abits(w);
        m = bb > m ? bb : m;
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) {
        if (mp) max_partial(mp, cav_, blockIdx.x, m);
        else atomic_max_bits(sc + mslot, m);
    }
}

// The max-norm's blocks meet on the cavity's slot (a batch) or, in a
// single-cavity context, spread over the partial words that the next
// convergence check combines into the slot.
static unsigned long long* bicg_max_words(Ctx* c) { return c->nb == 1 ? c->mpart : nullptr; }

static void bicg_max_final(Ctx* c, int mslot)
{
    if (c->nb != 1) return;
    c->defer_mf = true;
    launch_max_final(c, c->act, mslot);
}

void bicg_s_alpha(Ctx* c, const SegV& s, double* out, const double* r, const double* v, const double* part, int mslot)
{
    k_bicg_s_alpha<<<seg_grid(c, (long)kRedBlocks * c->nb), kT, 0, c->s>>>(s, out, r, v, c->sc, part, mslot,
                                                                           bicg_max_words(c));
    bicg_max_final(c, mslot);
}

// x = alpha ph + x and r = s (the cavities that finish at the half step)
__global__ void k_bicg_half_finish(SegV sv, double* __restrict__ x, const double* __restrict__ ph,
                                   double* __restrict__ r, const double* __restrict__ s, const double* __restrict__ scb)
{
    SEG_ENTER(sv, off, n);
    const double alpha = scb[(long)cav_ * S_NSLOT + S_ALPHA];
    SEG_LOOP(i, n)
    {
        x[off + i] = alpha * ph[off + i] + 1.0 * x[off + i];
        r[off + i] = s[off + i];
    }
}

void bicg_half_finish(Ctx* c, const SegV& s, double* x, const double* ph, double* r, const double* sv)
{
    k_bicg_half_finish<<<seg_grid(c, 8192L * c->nb), kT, 0, c->s>>>(s, x, ph, r, sv, c->sc);
}

// omega from the partials of t.t and t.s; x += alpha ph + omega sh; r = s -
// omega t with max|r| (into slot mslot, cleared by the partial pass, or
// into the partial words mp) and the partials of the next rho = r^.r into
// rpart.  Launched with
// kRedBlocks blocks per cavity, so those partials are the ones the partial
// pass would form.  Block 0 records t.t, t.s, omega and rho_prev = rho.
__global__ void k_bicg_full_update(SegV sv, double* __restrict__ x, const double* __restrict__ ph,
                                   const double* __restrict__ shv, double* __restrict__ r,
                                   const double* __restrict__ s, const double* __restrict__ t,
                                   double* __restrict__ scb, int mslot, const double* __restrict__ part,
                                   const double* __restrict__ rh, double* __restrict__ rpart,
                                   unsigned long long* __restrict__ mp)
{
    __shared__ double shd[kT / 64], bc;
    __shared__ unsigned long long sh[kT / 64];
    SEG_ENTER(sv, off, n);
    double* sc = scb + (long)cav_ * S_NSLOT;
    const double tt = dot_total(part, cav_, shd, &bc);
    const double ts = dot_total(part, (long)gridDim.y + cav_, shd, &bc);
    const double omega = bicg_omega(tt, ts), alpha = sc[S_ALPHA];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[S_DOT0] = tt;
        sc[S_DOT1] = ts;
        sc[S_OMEGA] = omega;
        sc[S_RHOP] = sc[S_RHO];
    }
    unsigned long long m = 0ull;
    double rho = 0.0;
    SEG_LOOP(i, n)
    {
        x[off + i] += alpha * ph[off + i] + omega * shv[off + i];
        const double v = s[off + i] - omega * t[off + i];
        r[off + i] = v;
        rho += rh[off + i] * v;
        const unsigned long long bb = abits(v);
        m = bb > m ? bb : m;
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) {
        if (mp) max_partial(mp, cav_, blockIdx.x, m);
        else atomic_max_bits(sc + mslot, m);
    }
    rho = block_sum(rho, shd);
    if (threadIdx.x == 0) rpart[(long)cav_ * kRedBlocks + blockIdx.x] = rho;
}

void bicg_full_update(Ctx* c, const SegV& s, double* x, const double* ph, const double* shv, double* r,
                      const double* sv, const double* t, int mslot, const double* part, const double* rh,
                      double* rpart)
{
    k_bicg_full_update<<<dim3(kRedBlocks, c->nb), kT, 0, c->s>>>(s, x, ph, shv, r, sv, t, c->sc, mslot, part, rh,
                                                                  rpart, bicg_max_words(c));
    bicg_max_final(c, mslot);
}

}  // namespace hb
