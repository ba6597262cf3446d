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
// padded to a multiple of 8 with zeros (16-byte loads in every precision of the ladder kernels).
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

// Gf holds ladder elements as rows (a,c), a in [a0, a0+na), and columns (b,d), b >= a0:
// (ac|bd) = Gf[((a-a0) v + c) ldf + (b-a0) v + d].  For a pair row (a,b) with b >= a, the v x v matrix
// M[c][d] = (ac|bd) is read in 32 x 32 tiles (c-tile <= d-tile) together with the mirrored tile M[d][c],
// both along their contiguous index, through LDS; the pair-block entries of the tile pair are written from
// the two.  One more block column writes the 8 padding columns of the row.
__global__ __launch_bounds__(256) void sa_form_kernel(const double* Gf, long long ldf, int a0, int v, double* Gp,
                                                      double* Gm, long long lp, long long lm) {
    __shared__ double T1[32][33], T2[32][33];
    const int r = blockIdx.y, a = a0 + r / v, b = r % v;
    if (b < a) return;
    const int nt = (v + 31) / 32, npr = nt * (nt + 1) / 2;
    double* gp = Gp + pidx(a, b, v) * lp;
    double* gm = a < b ? Gm + qidx(a, b, v) * lm : nullptr;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    if ((int)blockIdx.x == npr) {
        const long long np = (long long)v * (v + 1) / 2, nm = (long long)v * (v - 1) / 2;
        if (threadIdx.x < 8) {
            const int k = threadIdx.x;
            if (np + k < lp) gp[np + k] = 0.0;
            if (gm && nm + k < lm) gm[nm + k] = 0.0;
        }
        return;
    }
    int tc = 0, p = blockIdx.x;
    while (p >= nt - tc) { p -= nt - tc; ++tc; }
    const int td = tc + p;
    const double* M = Gf + ((long long)(a - a0) * v) * ldf + (long long)(b - a0) * v;  // M[c][d] = M[c * ldf + d]
    for (int i = ty; i < 32; i += 8) {
        const int c1 = tc * 32 + i, d1 = td * 32 + tx;  // tile (tc, td)
        T1[i][tx] = (c1 < v && d1 < v) ? M[(long long)c1 * ldf + d1] : 0.0;
        const int c2 = td * 32 + i, d2 = tc * 32 + tx;  // mirrored tile (td, tc)
        T2[i][tx] = (c2 < v && d2 < v) ? M[(long long)c2 * ldf + d2] : 0.0;
    }
    __syncthreads();
    for (int i = ty; i < 32; i += 8) {
        const int c = tc * 32 + i, d = td * 32 + tx;
        if (c >= v || d >= v || c > d) continue;
        const double g1 = T1[i][tx], g2 = T2[tx][i];  // M[c][d], M[d][c]
        gp[pidx(c, d, v)] = 0.5 * (g1 + g2);
        if (gm && c < d) gm[qidx(c, d, v)] = 0.5 * (g1 - g2);
    }
}

__global__ void sa_zero_rows_kernel(double* Gp, double* Gm, int v, long long lp, long long lm) {
    const long long np = (long long)v * (v + 1) / 2, nm = (long long)v * (v - 1) / 2;
    const long long n1 = (lp - np) * lp, n2 = (lm - nm) * lm;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n1 + n2;
         t += (long long)gridDim.x * blockDim.x) {
        if (t < n1) Gp[np * lp + t] = 0.0;
        else Gm[nm * lm + (t - n1)] = 0.0;
    }
}

inline dim3 grid_rows(long long rows, long long cols) {
    const long long gx = std::max<long long>(1, std::min<long long>((cols + NT - 1) / NT, 1024));
    const long long gy = std::max<long long>(1, std::min<long long>(rows, 65535));
    return dim3((unsigned)gx, (unsigned)gy);
}

inline unsigned grid_for(long long n) {
    long long b = (n + NT - 1) / NT;
    return (unsigned)std::max<long long>(1, std::min<long long>(b, 8192));
}
}  // namespace

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

void k_sa_form(const double* Gf, long long ldf, int a0, int na, int v, double* Gp, double* Gm, hipStream_t s) {
    if (g_dry || na <= 0 || v <= 0) return;
    if ((long long)na * v > 65535) fail(-1, "k_sa_form: chunk too large");
    const int nt = (v + 31) / 32, npr = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(sa_form_kernel, dim3((unsigned)(npr + 1), (unsigned)(na * v)), dim3(256), 0, s, Gf, ldf, a0, v,
                       Gp, Gm, sa_lp(v), sa_lm(v));
    LAUNCHCHK();
}

void k_sa_zero_pad_rows(double* Gp, double* Gm, int v, hipStream_t s) {
    if (g_dry || v <= 0) return;
    const long long lp = sa_lp(v), lm = sa_lm(v);
    const long long n = (lp - (long long)v * (v + 1) / 2) * lp + (lm - (long long)v * (v - 1) / 2) * lm;
    if (n <= 0) return;
    hipLaunchKernelGGL(sa_zero_rows_kernel, dim3(grid_for(n)), dim3(NT), 0, s, Gp, Gm, v, lp, lm);
    LAUNCHCHK();
}

}  // namespace adc3
