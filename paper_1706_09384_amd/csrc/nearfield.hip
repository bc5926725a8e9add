// Dense near-field tiles: every non-admissible leaf pair tau x sigma stores
// the full 3m x 3n block of Green's tensors (Section 3.1, O(mn) part), or of
// the collocation operator's entry blocks (Section 4).
//
// One workgroup per tile; threads walk the m*n point pairs with the row
// point fastest, so that each column of the column-major tile is written by
// consecutive lanes (three contiguous entries per lane).  Geometry is read
// from cluster-ordered float64 SoA arrays; the difference x - y, the distance
// and the phases are formed in float64.
#include "internal.hpp"

namespace hm {

template <typename R, bool Coll>
__global__ void __launch_bounds__(256) nearfield_kernel(Geometry g, GreenParams<R> gp,
                                                        const DenseBlk *__restrict__ blk,
                                                        cplx<R> *__restrict__ slab, R self_re,
                                                        R self_im, int32_t *__restrict__ err) {
    const DenseBlk b = blk[blockIdx.x];
    const int64_t ld = b.ld;   // padded (even) row count of the tile
    cplx<R> *tile = slab + b.off;
    const int32_t pairs = b.m * b.n;
    for (int32_t k = threadIdx.x; k < pairs; k += blockDim.x) {
        const int32_t i = k % b.m, j = k / b.m;
        const int32_t pi = b.rb + i, pj = b.cb + j;
        cplx<R> K[9];
        if constexpr (Coll) {
            colloc_block<R>(g, gp, pi, pj, K);
        } else if (g.same && pi == pj) {
#pragma unroll
            for (int e = 0; e < 9; ++e) K[e] = {R(0), R(0)};
            K[0] = K[4] = K[8] = {self_re, self_im};
        } else {
            const double dx = g.x[0][pi] - g.y[0][pj];
            const double dy = g.x[1][pi] - g.y[1][pj];
            const double dz = g.x[2][pi] - g.y[2][pj];
            if (dx == 0.0 && dy == 0.0 && dz == 0.0) {
                atomicAdd(err, 1);
#pragma unroll
                for (int e = 0; e < 9; ++e) K[e] = {R(0), R(0)};
            } else {
                R nx = 0, ny = 0, nz = 0;
                if (gp.kind == 1) {
                    nx = R(g.n[0][pj]);
                    ny = R(g.n[1][pj]);
                    nz = R(g.n[2][pj]);
                }
                green_block<R>(gp, dx, dy, dz, nx, ny, nz, K);
            }
        }
#pragma unroll
        for (int be = 0; be < 3; ++be) {
            cplx<R> *col = tile + (3 * (int64_t)j + be) * ld + 3 * i;
#pragma unroll
            for (int a = 0; a < 3; ++a) col[a] = K[3 * a + be];
        }
    }
}

template <typename R>
void launch_nearfield(const Geometry &g, const GreenParams<R> &gp, const DenseBlk *d_blk,
                      int32_t nblk, cplx<R> *slab, R self_re, R self_im, int32_t *d_err,
                      hipStream_t st, bool unbatched) {
    if (nblk == 0) return;
    const auto kern = g.mesh.tri ? nearfield_kernel<R, true> : nearfield_kernel<R, false>;
    if (unbatched) {
        // comparison baseline: one launch per tile
        for (int32_t i = 0; i < nblk; ++i)
            hipLaunchKernelGGL(kern, dim3(1), dim3(256), 0, st, g, gp, d_blk + i,
                               slab, self_re, self_im, d_err);
        HM_HIP_CHECK(hipGetLastError());
        return;
    }
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(256), 0, st, g, gp, d_blk, slab,
                       self_re, self_im, d_err);
    HM_HIP_CHECK(hipGetLastError());
}

template void launch_nearfield<float>(const Geometry &, const GreenParams<float> &,
                                      const DenseBlk *, int32_t, cplx<float> *, float, float,
                                      int32_t *, hipStream_t, bool);
template void launch_nearfield<double>(const Geometry &, const GreenParams<double> &,
                                       const DenseBlk *, int32_t, cplx<double> *, double, double,
                                       int32_t *, hipStream_t, bool);

}  // namespace hm
