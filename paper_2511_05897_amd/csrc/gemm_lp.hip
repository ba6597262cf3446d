// Reduced-precision GEMM on CDNA4 matrix cores with FP32 accumulation, FP64 output:
//   C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n)
// A is FP64 in HBM (converted while staging), B is stored in the reduced type.
//   prec 1: FP32 operands, v_mfma_f32_16x16x4f32   (BK = 16, 4 k-steps per slab)
//   prec 2: BF16 operands, v_mfma_f32_16x16x32_bf16 (BK = 32, 1 k-step per slab);
//           B is staged transposed in LDS so each lane reads its 8 consecutive k
//           as one 16-byte load.
// Accumulator layout of both FP32-output instructions: row 4*(l/16) + r, col l%16.
#include "internal.h"
#include <algorithm>

namespace adc3 {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

namespace {
constexpr int NT = 256;

template <int BM, int BN, int WM, int WN, int TAG>
__global__ __launch_bounds__(NT) void gemm_f32_kernel(GemmLP g) {
    constexpr int BK = 16;
    constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    constexpr int PA = (BM * BK + NT - 1) / NT, PB = (BN * BK + NT - 1) / NT;
    __shared__ float As[2][BM][BK + 1];
    __shared__ float Bs[2][BK][BN + 1];
    const int cz = blockIdx.z;
    const float* __restrict__ Bf = (const float*)g.B + cz * g.bB;
    const double* __restrict__ Ag = g.A + cz * g.bA;
    const float* __restrict__ Agf = g.Af ? g.Af + cz * g.bA : nullptr;
    double* __restrict__ Cg = g.C + cz * g.bC;
    const int K = (g.Klast >= 0 && cz == (int)gridDim.z - 1) ? g.Klast : g.K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)blockIdx.x * BN;
    const int wr = wave / WN, wc = wave % WN;
    const bool a_kc = (g.sAk == 1), b_nc = (g.sBn == 1);
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
    float ra[PA], rb[PB];
    auto fetch = [&](long long k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            long long m = m0 + ar[p], k = k0 + ak[p];
            ra[p] = (ar[p] >= 0 && m < g.M && k < K) ? (Agf ? Agf[m * g.sAm + k * g.sAk] : (float)Ag[m * g.sAm + k * g.sAk])
                                                    : 0.f;
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            long long kb = k0 + bk[p], n = n0 + bn[p];
            rb[p] = (bn[p] >= 0 && kb < K && n < g.N) ? Bf[kb * g.sBk + n * g.sBn] : 0.f;
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
    f4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int nslab = (K + BK - 1) / BK;
    if (nslab > 0) { fetch(0); stash(0); }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    const int rowbase = wr * (BM / WM), colbase = wc * (BN / WN);
    for (int s = 0; s < nslab; ++s) {
        const int buf = s & 1;
        if (s + 1 < nslab) fetch((long long)(s + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) af[i] = As[buf][rowbase + i * 16 + lr][kk + lk];
#pragma unroll
            for (int j = 0; j < TN; ++j) bf[j] = Bs[buf][kk + lk][colbase + j * 16 + lr];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
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
                long long row = m0 + rowbase + i * 16 + 4 * lk + r;
                long long col = n0 + colbase + j * 16 + lr;
                if (row < g.M && col < g.N) {
                    double* c = Cg + row * g.sCm + col * g.sCn;
                    double v = g.alpha * (double)acc[i][j][r];
                    *c = (g.beta == 0.0) ? v : v + g.beta * (*c);
                }
            }
}

template <int BM, int BN, int WM, int WN, int TAG>
__global__ __launch_bounds__(NT) void gemm_bf16_kernel(GemmLP g) {
    constexpr int BK = 32, PADK = 8;
    constexpr int TM = BM / WM / 16, TN = BN / WN / 16;
    constexpr int PA = (BM * BK + NT - 1) / NT, PB = (BN * BK + NT - 1) / NT;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][BM][BK + PADK];
    __shared__ __attribute__((aligned(16))) __bf16 Bt[2][BN][BK + PADK];  // transposed: [n][k]
    const int cz = blockIdx.z;
    const __bf16* __restrict__ Bh = (const __bf16*)g.B + cz * g.bB;
    const double* __restrict__ Ag = g.A + cz * g.bA;
    double* __restrict__ Cg = g.C + cz * g.bC;
    const int K = (g.Klast >= 0 && cz == (int)gridDim.z - 1) ? g.Klast : g.K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)blockIdx.x * BN;
    const int wr = wave / WN, wc = wave % WN;
    const bool a_kc = (g.sAk == 1), b_nc = (g.sBn == 1);
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
    __bf16 ra[PA], rb[PB];
    const __bf16 zero = (__bf16)0.f;
    auto fetch = [&](long long k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            long long m = m0 + ar[p], k = k0 + ak[p];
            ra[p] = (ar[p] >= 0 && m < g.M && k < K) ? (__bf16)(float)Ag[m * g.sAm + k * g.sAk] : zero;
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            long long kb = k0 + bk[p], n = n0 + bn[p];
            rb[p] = (bn[p] >= 0 && kb < K && n < g.N) ? Bh[kb * g.sBk + n * g.sBn] : zero;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (ar[p] >= 0) As[buf][ar[p]][ak[p]] = ra[p];
#pragma unroll
        for (int p = 0; p < PB; ++p)
            if (bn[p] >= 0) Bt[buf][bn[p]][bk[p]] = rb[p];
    };
    f4 acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const int nslab = (K + BK - 1) / BK;
    if (nslab > 0) { fetch(0); stash(0); }
    __syncthreads();
    const int lr = lane & 15, lk = lane >> 4;
    const int rowbase = wr * (BM / WM), colbase = wc * (BN / WN);
    for (int s = 0; s < nslab; ++s) {
        const int buf = s & 1;
        if (s + 1 < nslab) fetch((long long)(s + 1) * BK);
        bf8 af[TM], bfr[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = *(const bf8*)&As[buf][rowbase + i * 16 + lr][8 * lk];
#pragma unroll
        for (int j = 0; j < TN; ++j) bfr[j] = *(const bf8*)&Bt[buf][colbase + j * 16 + lr][8 * lk];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
        if (s + 1 < nslab) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                long long row = m0 + rowbase + i * 16 + 4 * lk + r;
                long long col = n0 + colbase + j * 16 + lr;
                if (row < g.M && col < g.N) {
                    double* c = Cg + row * g.sCm + col * g.sCn;
                    double v = g.alpha * (double)acc[i][j][r];
                    *c = (g.beta == 0.0) ? v : v + g.beta * (*c);
                }
            }
}

__global__ void to_f32_kernel(float* dst, const double* src, long long n) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        dst[t] = (float)src[t];
}
__global__ void to_bf16_kernel(__bf16* dst, const double* src, long long n) {
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        dst[t] = (__bf16)(float)src[t];
}
}  // namespace

static void launch_lp(const GemmLP& g, int prec, hipStream_t s, int tag, int nz) {
    const bool sk = g.M <= 16;
    dim3 grid(sk ? (g.N + 255) / 256 : (g.N + 79) / 80, sk ? (g.M + 15) / 16 : (g.M + 127) / 128, nz);
    if (prec == 1) {
        if (sk) hipLaunchKernelGGL((gemm_f32_kernel<16, 256, 1, 4, 0>), grid, dim3(NT), 0, s, g);
        else if (tag == 1) hipLaunchKernelGGL((gemm_f32_kernel<128, 80, 4, 1, 1>), grid, dim3(NT), 0, s, g);
        else hipLaunchKernelGGL((gemm_f32_kernel<128, 80, 4, 1, 0>), grid, dim3(NT), 0, s, g);
    } else if (prec == 2) {
        if (sk) hipLaunchKernelGGL((gemm_bf16_kernel<16, 256, 1, 4, 0>), grid, dim3(NT), 0, s, g);
        else if (tag == 1) hipLaunchKernelGGL((gemm_bf16_kernel<128, 80, 4, 1, 1>), grid, dim3(NT), 0, s, g);
        else hipLaunchKernelGGL((gemm_bf16_kernel<128, 80, 4, 1, 0>), grid, dim3(NT), 0, s, g);
    } else {
        fail(-1, "gemm_lp: unknown precision");
    }
    LAUNCHCHK();
}

void gemm_lp(const GemmLP& g, int prec, hipStream_t s, int tag) {
    if (g_dry) return;
    if (g.M <= 0 || g.N <= 0) return;
    const bool sk = g.M <= 16;
    const long long tiles = (long long)(sk ? (g.N + 255) / 256 : (g.N + 79) / 80) * (sk ? (g.M + 15) / 16 : (g.M + 127) / 128);
    const long long MN = (long long)g.M * g.N;
    if (tiles < 256 && g.K >= 4096 && g_gemm_scratch) {
        long long nchunk = std::min<long long>((g.K + 255) / 256, (2048 + tiles - 1) / tiles);
        nchunk = std::min<long long>(nchunk, g_gemm_scratch_n / std::max<long long>(MN, 1));
        nchunk = std::min<long long>(nchunk, 65535);
        if (nchunk >= 2) {
            const long long kc = (g.K + nchunk - 1) / nchunk;
            const long long nc = (g.K + kc - 1) / kc;
            GemmLP h = g;
            h.K = (int)kc;
            h.Klast = (int)(g.K - (nc - 1) * kc);
            h.alpha = 1.0; h.beta = 0.0;
            h.bA = kc * g.sAk; h.bB = kc * g.sBk; h.bC = MN;
            h.C = g_gemm_scratch; h.sCm = g.N; h.sCn = 1;
            launch_lp(h, prec, s, tag, (int)nc);
            splitk_reduce(g_gemm_scratch, (int)nc, g.M, g.N, g.alpha, g.beta, g.C, g.sCm, g.sCn, s);
            return;
        }
    }
    launch_lp(g, prec, s, tag, 1);
}

void k_to_lowp(void* dst, const double* src, long long n, int prec, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    if (!dst || !src) fail(-1, "k_to_lowp: NULL buffer");
    unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 8192);
    if (prec == 1) hipLaunchKernelGGL(to_f32_kernel, dim3(nb), dim3(256), 0, s, (float*)dst, src, n);
    else hipLaunchKernelGGL(to_bf16_kernel, dim3(nb), dim3(256), 0, s, (__bf16*)dst, src, n);
    LAUNCHCHK();
}

}  // namespace adc3
