// Formation of the stored ladder's pair blocks (see ladder_sa.hip for the blocks and their use):
// G+[(ab),(cd)] = ((ac|bd) + (ad|bc)) / 2 (a <= b, c <= d) and G-[(ab),(cd)] = ((ac|bd) - (ad|bc)) / 2
// (a < b, c < d), folded from ladder elements (ac|bd) that a GEMM over the DF factor produces for a chunk of
// the first virtual a; the padding rows and columns (to a multiple of 8) are zeroed.
#include "internal.h"
#include <algorithm>

namespace adc3 {

namespace {
__device__ inline long long pidx(int a, int b, int v) {  // a <= b
    return (long long)a * v - (long long)a * (a - 1) / 2 + (b - a);
}
__device__ inline long long qidx(int a, int b, int v) {  // a < b
    return (long long)a * (v - 1) - (long long)a * (a - 1) / 2 + (b - a - 1);
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

inline unsigned grid_for(long long n) {
    long long b = (n + 255) / 256;
    return (unsigned)std::max<long long>(1, std::min<long long>(b, 8192));
}
}  // namespace

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
    hipLaunchKernelGGL(sa_zero_rows_kernel, dim3(grid_for(n)), dim3(256), 0, s, Gp, Gm, v, lp, lm);
    LAUNCHCHK();
}

}  // namespace adc3
