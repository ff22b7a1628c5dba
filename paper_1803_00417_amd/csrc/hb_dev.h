// hb_dev.h -- device-side grid descriptor, indexing and boundary values for
// the HIP kernels of the Herschel-Bulkley step.  gfx950 (CDNA4), FP64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hb {

constexpr int kMaxLev = 24;
// largest dense coarsest system a hierarchy stops at (unknowns)
constexpr int kDenseMax = 128;
constexpr int kMaxTail = 8;   // levels handled by the single-workgroup coarse V-cycle

// Grid of one multigrid level, passed to kernels by value.
struct GridD {
    int dim;
    int n[3];          // cells per axis (1 on unused axes)
    double h;
    int per[3];        // 1 if the axis is periodic
    double wall_u[3][2][3];
};

// The same grid with its dimension fixed at compile time, for kernels
// instantiated per dimension (loops over the axes unroll, index arithmetic
// folds).  The wall velocities stay in the descriptor it was made from.
// Every grid helper below takes either kind.
template <int DIM>
struct GridS {
    static constexpr int dim = DIM;
    int n[3];
    double h;
    int per[3];
    const double (*wall_u)[2][3];
};

template <int DIM>
__device__ inline GridS<DIM> grid_s(const GridD& g)
{
    GridS<DIM> s;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s.n[a] = g.n[a];
        s.per[a] = g.per[a];
    }
    s.h = g.h;
    s.wall_u = g.wall_u;
    return s;
}

template <class G>
__host__ __device__ inline long ncells(const G& g) { return (long)g.n[0] * g.n[1] * g.n[2]; }

template <class G>
__host__ __device__ inline int nnode(const G& g, int a)
{
    return a >= g.dim ? 1 : (g.per[a] ? g.n[a] : g.n[a] + 1);
}
template <class G>
__host__ __device__ inline long nnodes(const G& g) { return (long)nnode(g, 0) * nnode(g, 1) * nnode(g, 2); }

template <class G>
__host__ __device__ inline int nface(const G& g, int a) { return g.per[a] ? g.n[a] : g.n[a] + 1; }

// extent along b of the face array of axis a
template <class G>
__host__ __device__ inline int fext(const G& g, int a, int b) { return b == a ? nface(g, a) : g.n[b]; }

template <class G>
__host__ __device__ inline long fcount(const G& g, int a)
{
    return (long)fext(g, a, 0) * fext(g, a, 1) * fext(g, a, 2);
}

template <class G>
__host__ __device__ inline long foffset(const G& g, int a)
{
    long o = 0;
    for (int b = 0; b < a; ++b) o += fcount(g, b);
    return o;
}

template <class G>
__host__ __device__ inline long cid(const G& g, int i, int j, int k)
{
    return ((long)k * g.n[1] + j) * g.n[0] + i;
}

template <class G>
__host__ __device__ inline long nid(const G& g, int i, int j, int k)
{
    return ((long)k * nnode(g, 1) + j) * nnode(g, 0) + i;
}

template <class G>
__host__ __device__ inline long fid(const G& g, int a, int i, int j, int k)
{
    return ((long)k * fext(g, a, 1) + j) * fext(g, a, 0) + i;
}

// Value of component c of a cell field at (i,j,k), which may lie up to two
// cells outside the box along one wall axis: wall ghosts are the odd
// reflection 2 u_b - q(mirror) (u_b = 0 when hom); periodic axes wrap.
template <bool HOM, class G>
__device__ inline double cval(const G& g, const double* __restrict__ q, int c, int i, int j, int k)
{
    int p[3] = {i, j, k};
    int oa = -1, side = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= g.dim) continue;
        const int n = g.n[a];
        int v = p[a];
        if (v >= 0 && v < n) continue;
        if (g.per[a]) {
            p[a] = v < 0 ? v + n : v - n;
        } else {
            oa = a;
            side = v < 0 ? 0 : 1;
            p[a] = v < 0 ? -1 - v : 2 * n - 1 - v;
        }
    }
    const double v = q[cid(g, p[0], p[1], p[2])];
    if (oa < 0) return v;
    const double ub = HOM ? 0.0 : g.wall_u[oa][side][c];
    return 2.0 * ub - v;
}

// wrap a cell index on periodic axes (callers pass indices at most one box
// length outside); returns false when the index lies beyond a wall
template <class G>
__device__ inline bool wrap(const G& g, int p[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= g.dim) continue;
        const int n = g.n[a];
        if (p[a] >= 0 && p[a] < n) continue;
        if (!g.per[a]) return false;
        p[a] = p[a] < 0 ? p[a] + n : p[a] - n;
    }
    return true;
}

// A uniform value (a per-cavity scalar slot such as dt) read with a vector
// load.  Scalar loads can only be waited for all together, so a scalar read
// from cold memory early in a kernel would hold back every later use of a
// kernel argument, and with it the issue of the data loads; a vector load is
// waited for with the data it travels with.
__device__ inline double vload(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// cell G moved into the box (per axis clamp): an in-range index for a cell
// whose value is then not used
template <class GR>
__device__ inline long cid_clamped(const GR& g, const int G[3])
{
    int p[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = G[a] < 0 ? 0 : (G[a] >= g.n[a] ? g.n[a] - 1 : G[a]);
    return cid(g, p[0], p[1], p[2]);
}

// Max-norm reductions work on the bit patterns of |v| as unsigned integers:
// they order like the values, and NaN (above +inf) propagates to the result.
__device__ inline unsigned long long abits(double v)
{
    return (unsigned long long)__double_as_longlong(fabs(v));
}

// (a maximum with 0 changes no word: blocks without values, such as those
// past the end of a small cavity of a batch, issue no atomic)
__device__ inline void atomic_max_bits(double* addr, unsigned long long v)
{
    if (v) atomicMax(reinterpret_cast<unsigned long long*>(addr), v);
}

// block-wide unsigned max (block of at most 1024 threads); valid in thread 0
__device__ inline unsigned long long block_umax(unsigned long long v, unsigned long long* sh)
{
    const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nt = blockDim.x * blockDim.y * blockDim.z;
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_down(v, off, 64);
        v = o > v ? o : v;
    }
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    if (t < 64) {
        v = (t < (nt + 63) / 64) ? sh[t] : 0ull;
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_down(v, off, 64);
            v = o > v ? o : v;
        }
    }
    __syncthreads();
    return v;
}

// block-wide sum in a fixed tree order; valid in thread 0
__device__ inline double block_sum(double v, double* sh)
{
    const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nt = blockDim.x * blockDim.y * blockDim.z;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    if (t < 64) {
        v = (t < (nt + 63) / 64) ? sh[t] : 0.0;
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    }
    __syncthreads();
    return v;
}

}  // namespace hb
