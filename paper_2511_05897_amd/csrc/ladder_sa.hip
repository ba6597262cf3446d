// The stored ladder in pair-symmetric and pair-antisymmetric blocks.
//
// The ladder sigma_z[a][b] = sum_cd (ac|bd) z[c][d] maps the part of z that is symmetric under
// c <-> d to a result symmetric under a <-> b, and the antisymmetric part to an antisymmetric
// result, because (ac|bd) = (bd|ac) for any real factorisation (pq|rs) = sum_Q B^Q_pq B^Q_rs.
// So the v^2 x v^2 matrix falls into two blocks over the pairs c <= d and c < d:
//   G+[(ab),(cd)] = ((ac|bd) + (ad|bc)) / 2   (a <= b, c <= d),  input w+ = z[c][d] + z[d][c] (c < d), z[c][c]
//   G-[(ab),(cd)] = ((ac|bd) - (ad|bc)) / 2   (a <  b, c <  d),  input w- = z[c][d] - z[d][c]
// and sigma[a][b] = (G+ w+)[(ab)] + (G- w-)[(ab)] for a < b, (G+ w+)[(ba)] - (G- w-)[(ba)] for a > b,
// (G+ w+)[(aa)] on the diagonal.  Both blocks are symmetric matrices; together they hold about half
// of the v^4 elements, so each application streams and multiplies half as much.  This is an exact
// rearrangement of the contraction (only the rounding order changes).
//
// Pair order is row-major over the upper triangle (a, then b).  Each block's leading dimension is
// padded to a multiple of 8 with zeros (16-byte loads in every precision of the ladder kernels).  This file
// holds the packing of the input rows, their k-major transpose (for the ladder kernels that copy both
// tiles straight into LDS) and the unpacking of the result; ladder_form.hip forms the blocks.
#include "internal.h"
#include <algorithm>

namespace adc3 {

namespace {
constexpr int NT = 256;

__device__ inline long long pidx(int a, int b, int v) {  // a <= b
    return (long long)a * v - (long long)a * (a - 1) / 2 + (b - a);
}
__device__ inline long long qidx(int a, int b, int v) {  // a < b
    return (long long)a * (v - 1) - (long long)a * (a - 1) / 2 + (b - a - 1);
}

// Rows m of z[m][v][v] (row stride ldz) -> w+[m][lp], w-[m][lm]; the padding columns are zeroed by
// the threads past M v^2.
__global__ void sa_pack_kernel(const double* z, long long ldz, int M, int v, double* Ws, double* Wa, long long lp,
                               long long lm) {
    const int vv = v * v;
    const long long np = (long long)v * (v + 1) / 2, nm = (long long)v * (v - 1) / 2;
    for (long long m = blockIdx.y; m < M; m += gridDim.y) {
        const double* zm = z + m * ldz;
        double* ws = Ws + m * lp;
        double* wa = Wa + m * lm;
        for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < vv + 8; r += gridDim.x * blockDim.x) {
            if (r < vv) {
                const int a = r / v, b = r - (r / v) * v;
                if (a > b) continue;
                if (a == b) {
                    ws[pidx(a, a, v)] = zm[r];
                } else {
                    const double x = zm[r], y = zm[b * v + a];
                    ws[pidx(a, b, v)] = x + y;
                    wa[qidx(a, b, v)] = x - y;
                }
            } else {
                const int k = r - vv;
                if (np + k < lp) ws[np + k] = 0.0;
                if (nm + k < lm) wa[nm + k] = 0.0;
            }
        }
    }
}

__global__ void sa_unpack_kernel(const double* Cs, const double* Ca, int M, int v, long long lp, long long lm,
                                 double* out, long long ldo) {
    const int vv = v * v;
    for (long long m = blockIdx.y; m < M; m += gridDim.y) {
        const double* cs = Cs + m * lp;
        const double* ca = Ca + m * lm;
        for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < vv; r += gridDim.x * blockDim.x) {
            const int a = r / v, b = r - (r / v) * v;
            double x;
            if (a == b) x = cs[pidx(a, a, v)];
            else if (a < b) x = cs[pidx(a, b, v)] + ca[qidx(a, b, v)];
            else x = cs[pidx(b, a, v)] - ca[qidx(b, a, v)];
            out[m * ldo + r] = x;
        }
    }
}

// 32 x 32 tiles through LDS (one padding column against bank conflicts); 256 threads, each moving
// 4 elements in and 4 out, both sides coalesced along the tile's rows
constexpr int TT = 32;
__global__ void transpose_kernel(const double* src, long long lds, int rows, long long cols, double* dst, long long ldd) {
    __shared__ double t[TT][TT + 1];
    const long long c0 = (long long)blockIdx.x * TT;
    const int r0 = blockIdx.y * TT;
    const int tx = threadIdx.x & (TT - 1), ty = threadIdx.x / TT;  // ty 0..7
#pragma unroll
    for (int q = 0; q < TT; q += 8) {
        const int r = r0 + ty + q;
        const long long c = c0 + tx;
        if (r < rows && c < cols) t[ty + q][tx] = src[(long long)r * lds + c];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TT; q += 8) {
        const long long c = c0 + ty + q;
        const int r = r0 + tx;
        if (r < rows && c < cols) dst[c * ldd + r] = t[tx][ty + q];
    }
}

inline dim3 grid_rows(long long rows, long long cols) {
    const long long gx = std::max<long long>(1, std::min<long long>((cols + NT - 1) / NT, 1024));
    const long long gy = std::max<long long>(1, std::min<long long>(rows, 65535));
    return dim3((unsigned)gx, (unsigned)gy);
}

}  // namespace

void k_transpose(const double* src, long long lds, int rows, long long cols, double* dst, long long ldd, hipStream_t s) {
    if (g_dry || rows <= 0 || cols <= 0) return;
    const long long gx = (cols + TT - 1) / TT, gy = (rows + TT - 1) / TT;
    if (gx > 0x7fffffffLL || gy > 65535) fail(-1, "transpose too large");
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, s, src, lds, rows, cols, dst, ldd);
    LAUNCHCHK();
}

long long sa_lp(int v) { return ((long long)v * (v + 1) / 2 + 7) / 8 * 8; }
long long sa_lm(int v) { return ((long long)v * (v - 1) / 2 + 7) / 8 * 8; }

void k_sa_pack(const double* z, long long ldz, int M, int v, double* Ws, double* Wa, hipStream_t s) {
    if (g_dry || M <= 0 || v <= 0) return;
    hipLaunchKernelGGL(sa_pack_kernel, grid_rows(M, (long long)v * v + 8), dim3(NT), 0, s, z, ldz, M, v, Ws, Wa, sa_lp(v),
                       sa_lm(v));
    LAUNCHCHK();
}

void k_sa_unpack(const double* Cs, const double* Ca, int M, int v, double* out, long long ldo, hipStream_t s) {
    if (g_dry || M <= 0 || v <= 0) return;
    hipLaunchKernelGGL(sa_unpack_kernel, grid_rows(M, (long long)v * v), dim3(NT), 0, s, Cs, Ca, M, v, sa_lp(v), sa_lm(v),
                       out, ldo);
    LAUNCHCHK();
}

}  // namespace adc3
