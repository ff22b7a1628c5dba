// hb_ws.hip -- transfers between the nodal pressure field and the cell grid
// of the warm-start network (2D), and the vector update of the warm start.
#include "hb_internal.h"

namespace hb {

// cell (i, j) takes scale times the mean of its four corner nodes (periodic
// axes wrap: node n is node 0)
__global__ void k_node_to_cell(GridD g, const double* __restrict__ v, double scale, float* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= g.n[0] || j >= g.n[1]) return;
    const int nx = nnode(g, 0), ny = nnode(g, 1);
    const int i1 = (i + 1 == nx) ? 0 : i + 1, j1 = (j + 1 == ny) ? 0 : j + 1;
    const double s = v[(long)j * nx + i] + v[(long)j * nx + i1] + v[(long)j1 * nx + i] + v[(long)j1 * nx + i1];
    out[(long)j * g.n[0] + i] = (float)(scale * 0.25 * s);
}

void launch_node_to_cell(Ctx* c, const GridD& g, const double* v, double scale, float* out)
{
    const dim3 blk(64, 4, 1);
    k_node_to_cell<<<grid3(g.n[0], g.n[1], 1, blk), blk, 0, c->s>>>(g, v, scale, out);
}

// node (i, j) takes the mean of the cells that share it
__global__ void k_cell_to_node(GridD g, const float* __restrict__ v, double* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int nx = nnode(g, 0), ny = nnode(g, 1);
    if (i >= nx || j >= ny) return;
    double s = 0.0;
    int cnt = 0;
    for (int dj = -1; dj <= 0; ++dj)
        for (int di = -1; di <= 0; ++di) {
            int p[3] = {i + di, j + dj, 0};
            if (!wrap(g, p)) continue;
            s += (double)v[(long)p[1] * g.n[0] + p[0]];
            ++cnt;
        }
    out[(long)j * nx + i] = s / (double)cnt;
}

void launch_cell_to_node(Ctx* c, const GridD& g, const float* v, double* out)
{
    const dim3 blk(64, 4, 1);
    k_cell_to_node<<<grid3(nnode(g, 0), nnode(g, 1), 1, blk), blk, 0, c->s>>>(g, v, out);
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ a, double s, long n)
{
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = x[i] + s * a[i];
}

void launch_axpy(Ctx* c, double* y, const double* x, const double* a, double s, long n)
{
    const long nb = (n + 255) / 256;
    k_axpy<<<(unsigned)(nb < 8192 ? nb : 8192), 256, 0, c->s>>>(y, x, a, s, n);
}

}  // namespace hb
