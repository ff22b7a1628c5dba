// hb_noalloc.hip -- the CFL time step without any allocation, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).
//
// The per-block partial maxima live in a file-scope device array of fixed
// size.  Its address on each device is taken once with hipGetSymbolAddress,
// with that device current, on the first call there; host code only ever
// passes that address (the array's name is a host-side stand-in).  Every call
// on a device shares its array: calls that overlap on one device (concurrent
// streams, threads) race on it.  Every partial a call reads was written by the
// same call, so nothing needs clearing between calls.
#include "hb_internal.h"

#include <mutex>

namespace hb {

static constexpr int kNaT = 256;          // threads per block
static constexpr int kNaPerThread = 16;   // values per thread
static constexpr long kNaMaxBlocks = 16384;
// largest velocity array (dim x cells values) one call accepts
static constexpr long kNaMaxValues = kNaMaxBlocks * kNaT * kNaPerThread;

static __device__ __align__(256) unsigned long long scratch[kNaMaxBlocks];

static std::mutex g_na_mu;
static unsigned long long* g_na_ptr[64];   // scratch's address per device

static unsigned long long* na_scratch(int* err)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { *err = 1; return nullptr; }
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) { *err = 1; return nullptr; }
        g_na_ptr[dev] = (unsigned long long*)p;
    }
    *err = 0;
    return g_na_ptr[dev];
}

// block b writes the largest |u| (bit pattern) of its kNaT * kNaPerThread values
__global__ void __launch_bounds__(kNaT) k_na_maxabs(const double* __restrict__ u, long n,
                                                    unsigned long long* __restrict__ part)
{
    __shared__ unsigned long long sh[kNaT / 64];
    const long base = (long)blockIdx.x * kNaT * kNaPerThread + threadIdx.x;
    unsigned long long m = 0ull;
#pragma unroll
    for (int t = 0; t < kNaPerThread; ++t) {
        const long i = base + (long)t * kNaT;
        if (i < n) {
            const unsigned long long b = abits(u[i]);
            m = b > m ? b : m;
        }
    }
    m = block_umax(m, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// one block: the largest partial, then dt = cfl h / max(U_wall, max|u|)
// (0 when both vanish, NaN for a non-finite velocity: inf - inf or NaN)
__global__ void __launch_bounds__(1024) k_na_dt(const unsigned long long* __restrict__ part, int nb, double ulid,
                                                double cfl, double h, double* __restrict__ dt)
{
    __shared__ unsigned long long sh[1024 / 64];
    unsigned long long m = 0ull;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) m = part[b] > m ? part[b] : m;
    m = block_umax(m, sh);
    if (threadIdx.x == 0) {
        const double um = __longlong_as_double((long long)m);
        const double mu = fmax(ulid, um);
        *dt = isfinite(um) ? (mu > 0.0 ? cfl * h / mu : 0.0) : um - um;
    }
}

}  // namespace hb

using namespace hb;

extern "C" int hb_cfl_dt_noalloc(const hb_grid* grid, double cfl, const double* u, double* dt_out, void* hip_stream)
{
    if (!grid || !u || !dt_out) {
        set_global_error("null argument");
        return HB_ERR_ARG;
    }
    if (const char* e = check_grid(grid)) {
        set_global_error(e);
        return HB_ERR_ARG;
    }
    if (!(cfl > 0.0)) {
        set_global_error("cfl must be positive");
        return HB_ERR_ARG;
    }
    long n = grid->dim;
    for (int a = 0; a < grid->dim; ++a) n *= grid->n[a];
    if (n > kNaMaxValues) {
        set_global_error("velocity larger than the static scratch allows (16384 blocks of 4096 values)");
        return HB_ERR_ARG;
    }
    double ulid = 0.0;
    for (int a = 0; a < grid->dim; ++a)
        for (int s = 0; s < 2 && grid->bc[a][0] != HB_BC_PERIODIC; ++s)
            for (int q = 0; q < 3; ++q) ulid = std::fmax(ulid, std::fabs(grid->wall_u[a][s][q]));
    int err = 0;
    unsigned long long* part = na_scratch(&err);
    if (err) {
        set_global_error("hipGetSymbolAddress of the static scratch failed");
        return HB_ERR_DEVICE;
    }
    const hipStream_t s = (hipStream_t)hip_stream;
    const int nb = (int)((n + (long)kNaT * kNaPerThread - 1) / ((long)kNaT * kNaPerThread));
    k_na_maxabs<<<nb, kNaT, 0, s>>>(u, n, part);
    k_na_dt<<<1, 1024, 0, s>>>(part, nb, ulid, cfl, grid->h, dt_out);
    if (hipGetLastError() != hipSuccess) {
        set_global_error("kernel launch failed");
        return HB_ERR_DEVICE;
    }
    return HB_OK;
}
