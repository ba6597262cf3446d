// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64), strided and batched.
//
// One workgroup = 4 wave64.  A BM x BN tile of C is split over the waves as a
// WM x WN grid; each wave accumulates (BM/WM) x (BN/WN) as 16x16 MFMA blocks.  A and
// B slabs (BM x 16, 16 x BN) are staged through LDS, double buffered: the next slab
// is fetched into registers while the current one feeds the matrix cores.  Global
// loads are coalesced along whichever operand dimension is contiguous.
//
// Tile shapes:
//   64x64   (2x2 waves)  general
//   16x256  (1x4 waves)  skinny: M <= 16 (Davidson linear combinations, 1p<->2p1h)
//   16x64   (1x4 waves)  M <= 16 and N <= 64 (K-chunked Gram blocks of the Davidson)
//   128x80  (4x1 waves)  sigma ladder: all (vector, occupied) rows in one tile, so the
//                        v^4 ladder matrix streams from HBM exactly once; 80 columns
//                        give 500 workgroups at v = 200 (2 per CU, one round)
//   128x128 (2x2 waves)  large square setup contractions
//
// MFMA f64 16x16x4 operand layout (lane l of a wave64):
//   A frag: A[row = l%16][k = l/16]   B frag: B[k = l/16][col = l%16]
//   D     : D[row = l/16 + 4*r][col = l%16] in accumulator element r = 0..3
#include "internal.h"
#include <algorithm>
#include <type_traits>

namespace adc3 {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int BK = 16, NT = 256;

template <int BM, int BN, int WM, int WN, int TAG>
__global__ __launch_bounds__(NT) void gemm_f64_kernel(Gemm g) {
    static_assert(WM * WN == 4, "four waves");
    constexpr int TM = BM / WM / 16, TN = BN / WN / 16;  // MFMA blocks per wave
    static_assert(TM >= 1 && TN >= 1 && (BM / WM) % 16 == 0 && (BN / WN) % 16 == 0, "tile");
    constexpr int PA = (BM * BK + NT - 1) / NT, PB = (BN * BK + NT - 1) / NT;
    __shared__ double As[2][BM][BK + 1];
    __shared__ double Bs[2][BK][BN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bz = blockIdx.z;
    const int b0 = bz % g.nb0, b1 = bz / g.nb0;
    const double* __restrict__ A = g.A + b0 * g.bA0 + b1 * g.bA1;
    const double* __restrict__ B = g.B + b0 * g.bB0 + b1 * g.bB1;
    double* __restrict__ C = g.C + b0 * g.bC0 + b1 * g.bC1;
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)blockIdx.x * BN;
    const int wr = wave / WN, wc = wave % WN;
    const bool a_kc = (g.sAk == 1), b_nc = (g.sBn == 1);
    const int K = (g.Klast >= 0 && b0 == g.nb0 - 1) ? g.Klast : g.K;

    int ar[PA], ak[PA], bk[PB], bn[PB];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
        int idx = tid + NT * p;
        if (idx >= BM * BK) { ar[p] = -1; ak[p] = 0; continue; }
        if (a_kc) { ar[p] = idx / BK; ak[p] = idx % BK; } else { ar[p] = idx % BM; ak[p] = idx / BM; }
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        int idx = tid + NT * p;
        if (idx >= BN * BK) { bn[p] = -1; bk[p] = 0; continue; }
        if (b_nc) { bn[p] = idx % BN; bk[p] = idx / BN; } else { bk[p] = idx % BK; bn[p] = idx / BK; }
    }
    double ra[PA], rb[PB];
    auto fetch = [&](long long k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            long long m = m0 + ar[p], k = k0 + ak[p];
            ra[p] = (ar[p] >= 0 && m < g.M && k < K) ? A[m * g.sAm + k * g.sAk] : 0.0;
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            long long kb = k0 + bk[p], n = n0 + bn[p];
            rb[p] = (bn[p] >= 0 && kb < K && n < g.N) ? B[kb * g.sBk + n * g.sBn] : 0.0;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (ar[p] >= 0) As[buf][ar[p]][ak[p]] = ra[p];
#pragma unroll
        for (int p = 0; p < PB; ++p)
            if (bn[p] >= 0) Bs[buf][bk[p]][bn[p]] = rb[p];
    };

    d4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const int nslab = (K + BK - 1) / BK;
    if (nslab > 0) {
        fetch(0);
        stash(0);
    }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    const int rowbase = wr * (BM / WM), colbase = wc * (BN / WN);
    for (int s = 0; s < nslab; ++s) {
        const int buf = s & 1;
        if (s + 1 < nslab) fetch((long long)(s + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = As[buf][rowbase + i * 16 + lr][kk + lk];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = Bs[buf][kk + lk][colbase + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (s + 1 < nslab) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                long long row = m0 + rowbase + i * 16 + lk + 4 * r;
                long long col = n0 + colbase + j * 16 + lr;
                if (row < g.M && col < g.N) {
                    double* c = C + row * g.sCm + col * g.sCn;
                    double v = g.alpha * acc[i][j][r];
                    *c = (g.beta == 0.0) ? v : v + g.beta * (*c);
                }
            }
}

// Deterministic: thread t sums chunks t, t+256, ... in order, then a fixed tree over threads.
__global__ void splitk_reduce_tree_kernel(const double* part, int nchunk, int M, int N, double alpha, double beta,
                                          double* C, long long sCm, long long sCn) {
    const long long MN = (long long)M * N, t = blockIdx.x;
    double acc = 0.0;
    for (int c = threadIdx.x; c < nchunk; c += blockDim.x) acc += part[(long long)c * MN + t];
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const long long m = t / N, n = t % N;
        double* cp = C + m * sCm + n * sCn;
        const double v = alpha * red[0];
        *cp = (beta == 0.0) ? v : v + beta * (*cp);
    }
}

__global__ void splitk_reduce_kernel(const double* part, int nchunk, int M, int N, double alpha, double beta,
                                     double* C, long long sCm, long long sCn) {
    long long MN = (long long)M * N;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < MN; t += (long long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int c = 0; c < nchunk; ++c) acc += part[(long long)c * MN + t];
        long long m = t / N, n = t % N;
        double* cp = C + m * sCm + n * sCn;
        double v = alpha * acc;
        *cp = (beta == 0.0) ? v : v + beta * (*cp);
    }
}

// Skinny products with both operands contiguous along K and a long K (the 1p <- 2p1h coupling product
// r2 U_z^T, M = vectors, N = virtuals, K = o v^2; Gram blocks of Davidson vectors):
//   part[c][m][n] = sum over k in chunk c of A[m][k] B[n][k],   M <= 16, N <= 256.
// No LDS: each wave loads its fragments straight from HBM.  One 16-k slab feeds four
// 16x16x4 MFMAs; the K order inside a slab is permuted so that a lane's four k are adjacent
// (k = k0 + 4q + j for lane group q = lane/16 at MFMA step j), which makes each lane's load
// one contiguous 32-byte run (two 16-byte loads) when the rows are 16-byte aligned.  The
// sum over k is the same set of products; only the order of the additions differs.  The four
// waves of a workgroup share its K chunk and split the N tiles (tile t on wave t % 4), so the
// U_z stream has no reduction inside the workgroup; the chunk partials are summed by
// splitk_reduce in chunk order (deterministic).  Rows and ks past the ends read as zero.
typedef double d2 __attribute__((ext_vector_type(2)));

template <bool VEC>
__global__ __launch_bounds__(NT) void abt_skinny_kernel(const double* __restrict__ A, long long lda,
                                                         const double* __restrict__ B, long long ldb, int M, int N,
                                                         long long K, long long kc, double* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const long long klo = (long long)blockIdx.x * kc;
    const long long khi = klo + kc < K ? klo + kc : K;
    const int nt = (N + 15) / 16;
    const bool arow = r < M;
    const double* Ar = A + (arow ? (long long)r * lda : 0);
    const double* Br[4];
    bool brow[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int n = 16 * (wave + 4 * i) + r;
        brow[i] = n < N;
        Br[i] = B + (brow[i] ? (long long)n * ldb : 0);
    }
    d4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    long long k0 = klo;
    if (VEC) {
        for (; k0 + 16 <= khi; k0 += 16) {
            const long long ko = k0 + 4 * q;
            d2 a0 = d2{0.0, 0.0}, a1 = d2{0.0, 0.0};
            if (arow) {
                a0 = *(const d2*)(Ar + ko);
                a1 = *(const d2*)(Ar + ko + 2);
            }
            d2 b0[4], b1[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                b0[i] = d2{0.0, 0.0}; b1[i] = d2{0.0, 0.0};
                if (wave + 4 * i < nt && brow[i]) {
                    b0[i] = *(const d2*)(Br[i] + ko);
                    b1[i] = *(const d2*)(Br[i] + ko + 2);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (wave + 4 * i >= nt) continue;  // uniform over the wave
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b0[i].x, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b0[i].y, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b1[i].x, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b1[i].y, acc[i], 0, 0, 0);
            }
        }
    }
    // the rest (all of the chunk on unaligned rows): element loads, k = k0 + 4j + q
    for (; k0 < khi; k0 += 16) {
        double a[4], b[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long k = k0 + 4 * j + q;
            a[j] = (arow && k < khi) ? Ar[k] : 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) b[i][j] = (wave + 4 * i < nt && brow[i] && k < khi) ? Br[i][k] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (wave + 4 * i >= nt) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b[i][j], acc[i], 0, 0, 0);
        }
    }
    double* P = part + (long long)blockIdx.x * M * N;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int n = 16 * (wave + 4 * i) + r;
        if (n >= N) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = q + 4 * e;
            if (m < M) P[(long long)m * N + n] = acc[i][e];
        }
    }
}

// Both 1p <-> 2p1h products of a sigma pass in one stream over U_z [a][k] (a < v <= 256 rows, k < K = o v^2):
//   part1[c][m][a] = sum over k in chunk c of r2[m][k] U[a][k]      (1p side, summed over chunks afterwards)
//   out2[m][k]     = sum_a r1[m][a] U[a][k]                          (2p1h side, written directly)
// for m < M <= 16.  A workgroup takes one K chunk; each 16-k slab of U is loaded once, as the MFMA
// fragments of the 1p product (waves split the 16-row tiles of a, as abt_skinny_kernel does), and
// parked in LDS; the four waves then read the slab back in the transposed fragment layout (contraction
// over a, MFMA steps of four a dealt out round-robin to the waves), the four partial 16 x 16 tiles are
// summed in LDS in wave order and the slab's out2 columns written.  Rows and ks past the ends read as
// zero.  Requires 16-byte aligned rows (even strides).  U_z in FP32 (the reduced-precision sigma passes) is
// widened to FP64 on load: the same fragments, and sums in FP64.
template <typename TU>
__global__ __launch_bounds__(NT, 3) void couple_fused_kernel(const TU* __restrict__ U, long long ldu, int v,
                                                          long long K, long long kc, const double* __restrict__ r2,
                                                          long long ld2, const double* __restrict__ r1, long long ld1,
                                                          int M, double* __restrict__ part1, double* __restrict__ out2,
                                                          long long ldo) {
    extern __shared__ double lds[];
    double* Us = lds;                       // [v][17]: the slab, row a, 16 k (+1 pad)
    double* Ps = lds + (long long)v * 17;   // [4][256]: the waves' out2 partial tiles [m][k]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, q = lane >> 4;
    const long long klo = (long long)blockIdx.x * kc;
    const long long khi = klo + kc < K ? klo + kc : K;
    const int nt = (v + 15) / 16, nsteps = (v + 3) / 4;
    const bool arow = r < M;
    const double* Ar = r2 + (arow ? (long long)r * ld2 : 0);
    const TU* Br[4];
    bool brow[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int a = 16 * (wave + 4 * i) + r;
        brow[i] = a < v;
        Br[i] = U + (brow[i] ? (long long)a * ldu : 0);
    }
    // r1 fragments of this wave's contraction steps s = wave + 4 i: lane (m = r, q) holds r1[m][4 s + q]
    double f1[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int a = 4 * (wave + 4 * i) + q;
        f1[i] = (arow && a < v) ? r1[(long long)r * ld1 + a] : 0.0;
    }
    d4 acc[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};
    for (long long k0 = klo; k0 < khi; k0 += 16) {
        const long long ko = k0 + 4 * q;
        const bool full = k0 + 16 <= khi;
        double a4[4], b4[4][4];
        if (full) {
            d2 x0 = d2{0.0, 0.0}, x1 = d2{0.0, 0.0};
            if (arow) {
                x0 = *(const d2*)(Ar + ko);
                x1 = *(const d2*)(Ar + ko + 2);
            }
            a4[0] = x0.x; a4[1] = x0.y; a4[2] = x1.x; a4[3] = x1.y;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if constexpr (std::is_same<TU, float>::value) {
                    // FP32 U_z: one 16-byte load of four k, widened to FP64
                    float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (wave + 4 * i < nt && brow[i]) y = *(const float4*)(Br[i] + ko);
                    b4[i][0] = y.x; b4[i][1] = y.y; b4[i][2] = y.z; b4[i][3] = y.w;
                } else {
                    d2 y0 = d2{0.0, 0.0}, y1 = d2{0.0, 0.0};
                    if (wave + 4 * i < nt && brow[i]) {
                        y0 = *(const d2*)(Br[i] + ko);
                        y1 = *(const d2*)(Br[i] + ko + 2);
                    }
                    b4[i][0] = y0.x; b4[i][1] = y0.y; b4[i][2] = y1.x; b4[i][3] = y1.y;
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long long k = ko + j;
                a4[j] = (arow && k < khi) ? Ar[k] : 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) b4[i][j] = (wave + 4 * i < nt && brow[i] && k < khi) ? Br[i][k] : 0.0;
            }
        }
        // 1p product (k = ko + j at MFMA step j) and the slab into LDS
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (wave + 4 * i >= nt) continue;  // uniform over the wave
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a4[j], b4[i][j], acc[i], 0, 0, 0);
            if (brow[i]) {
                double* u = Us + (long long)(16 * (wave + 4 * i) + r) * 17 + 4 * q;
#pragma unroll
                for (int j = 0; j < 4; ++j) u[j] = b4[i][j];
            }
        }
        __syncthreads();
        // 2p1h product over a: D[m][k] += r1[m][a] U[a][k], lane (k = r, a = 4 s + q); the slab's fragments
        // read eight steps at a time, two accumulators (even and odd steps) summed at the end
        d4 d0 = d4{0.0, 0.0, 0.0, 0.0}, d1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 16; h += 8) {
            if (wave + 4 * h >= nsteps) break;  // uniform over the wave
            double bb[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int st = wave + 4 * (h + i), a = 4 * st + q;
                bb[i] = (st < nsteps && a < v) ? Us[a * 17 + r] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                if (wave + 4 * (h + i) < nsteps) d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(f1[h + i], bb[i], d0, 0, 0, 0);
                if (wave + 4 * (h + i + 1) < nsteps)
                    d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(f1[h + i + 1], bb[i + 1], d1, 0, 0, 0);
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) Ps[wave * 256 + (q + 4 * e) * 16 + r] = d0[e] + d1[e];
        __syncthreads();
        {
            const int m = tid >> 4, kk = tid & 15;
            const long long k = k0 + kk;
            if (m < M && k < khi)
                out2[(long long)m * ldo + k] =
                    ((Ps[m * 16 + kk] + Ps[256 + m * 16 + kk]) + Ps[512 + m * 16 + kk]) + Ps[768 + m * 16 + kk];
        }
    }
    double* P = part1 + (long long)blockIdx.x * M * v;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int a = 16 * (wave + 4 * i) + r;
        if (a >= v) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = q + 4 * e;
            if (m < M) P[(long long)m * v + a] = acc[i][e];
        }
    }
}

enum Shape { SH_64x64 = 0, SH_16x256 = 1, SH_128x80 = 2, SH_128x128 = 3, SH_16x64 = 4 };
inline int tile_m(int sh) { return sh == SH_64x64 ? 64 : (sh == SH_16x256 || sh == SH_16x64) ? 16 : 128; }
inline int tile_n(int sh) {
    return sh == SH_64x64 ? 64 : sh == SH_16x256 ? 256 : sh == SH_128x80 ? 80 : sh == SH_16x64 ? 64 : 128;
}

int pick_shape(const Gemm& g, int tag) {
    if (tag == 1) return SH_128x80;
    if (g.M <= 16 && g.N <= 64) return SH_16x64;
    if (g.M <= 16) return SH_16x256;
    long long t128 = (long long)((g.M + 127) / 128) * ((g.N + 127) / 128);
    if (g.M >= 128 && g.N >= 128 && t128 * g.nb0 * g.nb1 >= 512) return SH_128x128;
    return SH_64x64;
}

void launch_tiles(const Gemm& g, hipStream_t s, int tag, long long nb, int sh) {
    const int bm = tile_m(sh), bn = tile_n(sh);
    dim3 grid((unsigned)((g.N + bn - 1) / bn), (unsigned)((g.M + bm - 1) / bm), (unsigned)nb);
    if (grid.y > 65535) fail(-1, "gemm: M too large");
    switch (sh) {
        case SH_16x256:
            hipLaunchKernelGGL((gemm_f64_kernel<16, 256, 1, 4, 0>), grid, dim3(NT), 0, s, g);
            break;
        case SH_16x64:
            hipLaunchKernelGGL((gemm_f64_kernel<16, 64, 1, 4, 0>), grid, dim3(NT), 0, s, g);
            break;
        case SH_128x80:
            if (tag == 1)  // sigma ladder: own symbol for profiling
                hipLaunchKernelGGL((gemm_f64_kernel<128, 80, 4, 1, 1>), grid, dim3(NT), 0, s, g);
            else
                hipLaunchKernelGGL((gemm_f64_kernel<128, 80, 4, 1, 0>), grid, dim3(NT), 0, s, g);
            break;
        case SH_128x128:
            hipLaunchKernelGGL((gemm_f64_kernel<128, 128, 2, 2, 0>), grid, dim3(NT), 0, s, g);
            break;
        default:
            hipLaunchKernelGGL((gemm_f64_kernel<64, 64, 2, 2, 0>), grid, dim3(NT), 0, s, g);
    }
    LAUNCHCHK();
}
}  // namespace

void splitk_reduce(const double* part, int nchunk, int M, int N, double alpha, double beta, double* C,
                   long long sCm, long long sCn, hipStream_t s) {
    long long MN = (long long)M * N;
    if (MN <= 32768 && nchunk >= 64) {
        // few outputs, many chunks: one block per output, chunks spread over its threads
        hipLaunchKernelGGL(splitk_reduce_tree_kernel, dim3((unsigned)MN), dim3(256), 0, s, part, nchunk, M, N, alpha,
                           beta, C, sCm, sCn);
    } else {
        unsigned gb = (unsigned)std::min<long long>((MN + 255) / 256, 4096);
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(gb), dim3(256), 0, s, part, nchunk, M, N, alpha, beta, C, sCm,
                           sCn);
    }
    LAUNCHCHK();
}

long long abt_skinny_chunks(int M, int N, long long K, long long partial_elems) {
    if (M < 1 || M > 16 || N < 1 || N > 256 || K < 256) return 0;
    // about 1024 workgroups (all resident at once at the kernel's occupancy: 4 per CU, 16 waves), each over a K chunk
    // of at least 256.  At o=20 v=200 the coupling product takes 257 us (5.0 TB/s over U_z; 295 us on the
    // LDS-staged split-K GEMM); requesting the next slab before the current slab's MFMAs (3 workgroups per
    // CU, 768 of them) measured no faster there and slower on the Gram blocks (64 against 52 us).
    long long nch = std::min<long long>(1024, K / 256);
    nch = std::min<long long>(nch, partial_elems / ((long long)M * N));
    return nch >= 2 ? nch : 0;
}

long long abt_skinny(int M, int N, long long K, const double* A, long long lda, const double* B, long long ldb,
                     double* part, long long partial_elems, hipStream_t s) {
    const long long want = abt_skinny_chunks(M, N, K, partial_elems);
    if (want == 0) return 0;
    const long long kc = ((K + want - 1) / want + 15) / 16 * 16;
    const long long nch = (K + kc - 1) / kc;
    const bool vec = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && lda % 2 == 0 && ldb % 2 == 0;
    if (vec)
        hipLaunchKernelGGL((abt_skinny_kernel<true>), dim3((unsigned)nch), dim3(NT), 0, s, A, lda, B, ldb, M, N, K, kc,
                           part);
    else
        hipLaunchKernelGGL((abt_skinny_kernel<false>), dim3((unsigned)nch), dim3(NT), 0, s, A, lda, B, ldb, M, N, K, kc,
                           part);
    LAUNCHCHK();
    return nch;
}

template <typename TU>
static long long couple_fused_t(int M, int v, long long K, const TU* U, long long ldu, const double* r2, long long ld2,
                                const double* r1, long long ld1, double* out2, long long ldo, double* part1,
                                long long partial_elems, hipStream_t s) {
    if (M < 1 || M > 16 || v < 1 || v > 256 || K < 256) return 0;
    if ((uintptr_t)U % 16 || (uintptr_t)r2 % 16 || ldu % (16 / (long long)sizeof(TU)) || ld2 % 2) return 0;
    long long want = std::min<long long>(768, K / 256);
    want = std::min<long long>(want, partial_elems / ((long long)M * v));
    if (want < 2) return 0;
    const long long kc = ((K + want - 1) / want + 15) / 16 * 16;
    const long long nch = (K + kc - 1) / kc;
    const size_t lds = ((size_t)v * 17 + 4 * 256) * sizeof(double);
    hipLaunchKernelGGL(couple_fused_kernel<TU>, dim3((unsigned)nch), dim3(NT), lds, s, U, ldu, v, K, kc, r2, ld2, r1,
                       ld1, M, part1, out2, ldo);
    LAUNCHCHK();
    return nch;
}

long long couple_fused(int M, int v, long long K, const double* U, long long ldu, const double* r2, long long ld2,
                       const double* r1, long long ld1, double* out2, long long ldo, double* part1,
                       long long partial_elems, hipStream_t s) {
    return couple_fused_t(M, v, K, U, ldu, r2, ld2, r1, ld1, out2, ldo, part1, partial_elems, s);
}

long long couple_fused32(int M, int v, long long K, const float* U, long long ldu, const double* r2, long long ld2,
                         const double* r1, long long ld1, double* out2, long long ldo, double* part1,
                         long long partial_elems, hipStream_t s) {
    return couple_fused_t(M, v, K, U, ldu, r2, ld2, r1, ld1, out2, ldo, part1, partial_elems, s);
}

thread_local double* g_gemm_scratch = nullptr;
thread_local long long g_gemm_scratch_n = 0;

GemmScratch::GemmScratch(Arena& ws, long long n) : prev(g_gemm_scratch), prev_n(g_gemm_scratch_n) {
    double* p = ws.take<double>((size_t)n);
    g_gemm_scratch = p;
    g_gemm_scratch_n = p ? n : 0;
}
GemmScratch::~GemmScratch() {
    g_gemm_scratch = prev;
    g_gemm_scratch_n = prev_n;
}

static void gemm_impl(const Gemm& g, hipStream_t s, int tag, int kmin_split);

void gemm(const Gemm& g, hipStream_t s, int tag) { gemm_impl(g, s, tag, 4096); }

void gemm_split(const Gemm& g, hipStream_t s, int tag) { gemm_impl(g, s, tag, 512); }

static void gemm_impl(const Gemm& g, hipStream_t s, int tag, int kmin_split) {
    if (g_dry) return;
    if (g.M <= 0 || g.N <= 0) return;
    long long nb = (long long)g.nb0 * g.nb1;
    if (nb <= 0) return;
    // K <= 0 is valid: the kernel then writes C = beta*C.
    if (nb > 65535) fail(-1, "gemm: too many batches");
    const int sh = pick_shape(g, tag);
    // large single GEMMs with A k-major and B, C row-major: the ladder kernel that copies both tiles
    // straight into LDS, when K fits one of its chunks
    if (sh == SH_128x128 && nb == 1 && g.sAm == 1 && g.sBn == 1 && g.sCn == 1 &&
        ladder_t_supported(g.M, g.N, g.K, g.A, g.sAk, g.B, g.sBk)) {
        const int nmin = ladder_t_min_chunks(g.K, g.sAk, g.sBk);
        if (nmin == 1 &&
            ladder_gemm_t(g.M, g.N, g.K, g.alpha, g.A, g.sAk, g.B, g.sBk, g.beta, g.C, g.sCm, 1, nullptr, 0, s, 2))
            return;
        if (nmin > 1) {
            // K past the kernel's 32-bit offsets in one launch: consecutive K ranges of one chunk each (a
            // multiple of 64 rows), accumulated into C in order
            const long long kc = ((g.K + nmin - 1) / nmin + 63) / 64 * 64;
            bool ok = true;
            for (long long k0 = 0; k0 < g.K && ok; k0 += kc) {
                const int kk = (int)std::min<long long>(kc, g.K - k0);
                ok = ladder_t_supported(g.M, g.N, kk, g.A + k0 * g.sAk, g.sAk, g.B + k0 * g.sBk, g.sBk) &&
                     ladder_t_min_chunks(kk, g.sAk, g.sBk) == 1;
            }
            if (ok) {
                for (long long k0 = 0; k0 < g.K; k0 += kc) {
                    const int kk = (int)std::min<long long>(kc, g.K - k0);
                    ladder_gemm_t(g.M, g.N, kk, g.alpha, g.A + k0 * g.sAk, g.sAk, g.B + k0 * g.sBk, g.sBk,
                                  k0 == 0 ? g.beta : 1.0, g.C, g.sCm, 1, nullptr, 0, s, 2);
                }
                return;
            }
        }
    }
    // large single GEMMs with both operands contiguous along their tile rows: the ladder kernel's
    // tile (whole-M row blocks, 2 workgroups per CU, 16-byte loads) without splitting K
    if (sh == SH_128x128 && nb == 1 && g.sAk == 1 && g.sBn == 1 && g.sCn == 1 &&
        ladder_supported(g.M, g.N, g.K, g.A, g.sAm, g.B, g.sBk, g.C, g.sCm)) {
        ladder_gemm(g.M, g.N, g.K, g.alpha, g.A, g.sAm, g.B, g.sBk, g.beta, g.C, g.sCm, 1, nullptr, 0, s, 2);
        return;
    }
    // skinny products with both operands contiguous along a long K: the fragment-streaming kernel
    if (nb == 1 && g.sAk == 1 && g.sBk == 1 && g.K >= kmin_split && g_gemm_scratch && g.M <= 16 && g.N <= 256) {
        const long long nch = abt_skinny(g.M, g.N, g.K, g.A, g.sAm, g.B, g.sBn, g_gemm_scratch, g_gemm_scratch_n, s);
        if (nch > 0) {
            splitk_reduce(g_gemm_scratch, (int)nch, g.M, g.N, g.alpha, g.beta, g.C, g.sCm, g.sCn, s);
            return;
        }
    }
    const long long tiles = (long long)((g.N + tile_n(sh) - 1) / tile_n(sh)) * ((g.M + tile_m(sh) - 1) / tile_m(sh));
    const long long MN = (long long)g.M * g.N;
    // few output tiles and a long K: cut K into chunks (one batch each), then sum the
    // partial tiles in a fixed order (deterministic)
    if (nb == 1 && tiles < 256 && g.K >= kmin_split && g_gemm_scratch) {
        // about 512 workgroups (2 per CU): at o=20 v=200 the 1p coupling product (one tile, K = o v^2)
        // takes 291 + 8 us (GEMM + reduction) with 512 chunks, 306 + 21 us with 2048, 385 + 6 us with 256
        long long nchunk = std::min<long long>((g.K + 255) / 256, (512 + tiles - 1) / tiles);
        nchunk = std::min<long long>(nchunk, g_gemm_scratch_n / std::max<long long>(MN, 1));
        nchunk = std::min<long long>(nchunk, 65535);
        if (nchunk >= 2) {
            const long long kc = (g.K + nchunk - 1) / nchunk;
            const long long nc = (g.K + kc - 1) / kc;
            const long long last = g.K - (nc - 1) * kc;
            Gemm h = g;
            h.K = (int)kc;
            h.Klast = (int)last;
            h.alpha = 1.0; h.beta = 0.0;
            h.bA0 = kc * g.sAk; h.bB0 = kc * g.sBk;
            h.C = g_gemm_scratch; h.sCm = g.N; h.sCn = 1; h.bC0 = MN;
            h.nb0 = (int)nc; h.nb1 = 1;
            launch_tiles(h, s, tag, nc, sh);
            splitk_reduce(g_gemm_scratch, (int)nc, g.M, g.N, g.alpha, g.beta, g.C, g.sCm, g.sCn, s);
            return;
        }
    }
    launch_tiles(g, s, tag, nb, sh);
}

void gemm_rm(int M, int N, int K, double alpha, const double* A, long long lda, bool transA,
             const double* B, long long ldb, bool transB, double beta, double* C, long long ldc,
             hipStream_t s, int tag) {
    Gemm g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.sAm = transA ? 1 : lda; g.sAk = transA ? lda : 1;
    g.B = B; g.sBk = transB ? 1 : ldb; g.sBn = transB ? ldb : 1;
    g.C = C; g.sCm = ldc; g.sCn = 1;
    g.alpha = alpha; g.beta = beta;
    gemm(g, s, tag);
}

}  // namespace adc3
