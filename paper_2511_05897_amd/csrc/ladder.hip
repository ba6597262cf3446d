// The sigma ladder as dedicated matrix-core kernels (FP64, and FP32 / BF16 operands).
//
//   C[m][n] = alpha * sum_k Z[m][k] G[k][n] + beta * C[m][n]
//
// m runs over (vector, occupied) pairs (a few hundred at most), k and n over virtual
// pairs, and G is one of the stored ladder's two symmetric blocks:
// G+[(cd)][(ab)] = ((ac|bd) + (ad|bc))/2 over c<=d, a<=b, or G-[(cd)][(ab)] =
// ((ac|bd) - (ad|bc))/2 over c<d, a<b (each side padded to a multiple of 8).  The
// same kernels serve the setup's large contractions (tag 2).
// The kernel is shaped by three facts of this contraction on CDNA4:
//   * all m rows fit one tile (TM blocks of 16 rows), so G streams from HBM exactly once;
//   * FP64 MFMA is the bound (2 flops per G element per row, >= 20 rows), so the tile
//     keeps 2 workgroups per CU (<= 256 registers a lane) to hide load latency across
//     workgroups rather than within one;
//   * K is split into chunks (deterministic partial sums, reduced in a fixed order) to
//     give >= 4 workgroups per CU slot; with a multiple of 8 chunks, the workgroups that
//     one XCD runs together share one chunk of Z in that XCD's L2.
// The chunk count and the row tiling (the default, or one more, shorter row tile) are chosen
// per shape by measurement on first use (ladder_tuned_chunks).
// Two FP64 forms: ladder_f64_kernel takes Z row-major and stages both tiles through
// registers into double-buffered LDS (16-byte loads, the Z tile transposed to [k][m] on the
// way, so that the 16 lanes of a fragment read 16 consecutive words); ladder_f64t_kernel
// takes Z k-major ([k][m], as G is [k][n]) and copies both tiles straight from HBM into LDS
// with buffer loads (its own comment below).  The sigma pass uses the second for row tiles
// of three or more 16-row blocks (33 rows and up).
//
// MFMA f64 16x16x4 (lane l of a wave64): A frag A[l%16][l/16], B frag B[l/16][l%16],
// accumulator element r holds D[l/16 + 4r][l%16].
#include "internal.h"
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

namespace adc3 {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

namespace {
constexpr int LBK = 16, LNT = 256, LTN = 2, LBN = 4 * 16 * LTN;  // 128 columns, 4 waves side by side
constexpr int APAD = 1, BPAD = 2;

struct LadderArgs {
    const double* Z; long long ldz;
    const double* G; long long ldg;
    double* C; long long ldc;
    double* P;  // partials [nchunk][M][N] when nchunk > 1
    int M, N, K, Kc, ntn, nchunk;
    double alpha, beta;
};

// TAG 1 marks the tuner's trial launches, TAG 2 other large GEMMs on this tile (separate symbols
// for profilers).
template <int TM, int TAG>
__global__ __launch_bounds__(LNT, 2) void ladder_f64_kernel(LadderArgs g) {
    constexpr int BM = 16 * TM;
    constexpr int PA = (BM * (LBK / 2) + LNT - 1) / LNT;  // 16-byte A loads per thread
    constexpr int PB = (LBK * (LBN / 2)) / LNT;            // 16-byte B loads per thread
    __shared__ __attribute__((aligned(16))) double As[2][LBK][BM + APAD];  // transposed: [k][m]
    __shared__ __attribute__((aligned(16))) double Bs[2][LBK][LBN + BPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    // block -> (chunk, column tile), XCD-grouped when the chunk count allows it
    const int b = blockIdx.x;
    int chunk, nt;
    if ((g.nchunk & 7) == 0) {
        const int q = b >> 3;
        chunk = (q / g.ntn) * 8 + (b & 7);
        nt = q % g.ntn;
    } else {
        chunk = b / g.ntn;
        nt = b % g.ntn;
    }
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)nt * LBN;
    const int kb = chunk * g.Kc, ke = std::min(g.K, kb + g.Kc);
    // per-thread load slots
    int arow[PA], akq[PA], bkr[PB], bnq[PB];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
        const int idx = tid + LNT * p;
        arow[p] = idx < BM * (LBK / 2) ? idx / (LBK / 2) : -1;
        akq[p] = idx % (LBK / 2);
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int idx = tid + LNT * p;
        bkr[p] = idx / (LBN / 2);
        bnq[p] = idx % (LBN / 2);
    }
    // Every load is issued, from an address clamped into the operands; the elements outside
    // the tile or the chunk are zeroed when the slab is written to LDS.  Without branches around
    // the loads the compiler can wait for one register set while the next is still in flight.
    const d2v z2 = {0.0, 0.0};
    auto fetch = [&](int k0, d2v(&ra)[PA], d2v(&rb)[PB]) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const long long m = std::min(m0 + std::max(arow[p], 0), (long long)g.M - 1);
            const int k = std::min(k0 + 2 * akq[p], g.K - 2);
            ra[p] = *(const d2v*)(g.Z + m * g.ldz + k);
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int k = std::min(k0 + bkr[p], g.K - 1);
            const long long n = std::min(n0 + 2 * bnq[p], (long long)g.N - 2);
            rb[p] = *(const d2v*)(g.G + (long long)k * g.ldg + n);
        }
    };
    auto stash = [&](int buf, int k0, const d2v(&ra)[PA], const d2v(&rb)[PB]) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (arow[p] >= 0) {
                const d2v x = (m0 + arow[p] < g.M && k0 + 2 * akq[p] < ke) ? ra[p] : z2;
                As[buf][2 * akq[p]][arow[p]] = x.x;
                As[buf][2 * akq[p] + 1][arow[p]] = x.y;
            }
#pragma unroll
        for (int p = 0; p < PB; ++p)
            *(d2v*)&Bs[buf][bkr[p]][2 * bnq[p]] = (k0 + bkr[p] < ke && n0 + 2 * bnq[p] < g.N) ? rb[p] : z2;
    };
    d4v acc[TM][LTN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
    const int cb = wave * (16 * LTN);
    auto compute = [&](int buf) {
#pragma unroll
        for (int kk = 0; kk < LBK; kk += 4) {
            double bf[LTN];
#pragma unroll
            for (int j = 0; j < LTN; ++j) bf[j] = Bs[buf][kk + lk][cb + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const double af = As[buf][kk + lk][16 * i + lr];
#pragma unroll
                for (int j = 0; j < LTN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf[j], acc[i][j], 0, 0, 0);
            }
        }
    };
    const int nslab = (ke - kb + LBK - 1) / LBK;
    // two slabs in flight in two register sets: slab s+2 is fetched while slab s is multiplied
    // and slab s+1 (fetched one slab earlier) is written to LDS after it
    d2v ra0[PA], rb0[PB], ra1[PA], rb1[PB];
    fetch(kb, ra0, rb0);
    fetch(kb + LBK, ra1, rb1);
    stash(0, kb, ra0, rb0);
    __syncthreads();
    auto step = [&](int s, d2v(&rc)[PA], d2v(&rbc)[PB], const d2v(&rn)[PA], const d2v(&rbn)[PB]) {
        fetch(kb + (s + 2) * LBK, rc, rbc);
        compute(s & 1);
        stash((s & 1) ^ 1, kb + (s + 1) * LBK, rn, rbn);
        __syncthreads();
    };
    int s = 0;
    for (; s + 1 < nslab; s += 2) {  // no branch inside the body, so no wait on the set in flight
        step(s, ra0, rb0, ra1, rb1);
        step(s + 1, ra1, rb1, ra0, rb0);
    }
    if (s < nslab) step(s, ra0, rb0, ra1, rb1);
    // epilogue: partial sums, or the final alpha/beta update when K is not split
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = m0 + 16 * i + lk + 4 * r;
                const long long col = n0 + cb + 16 * j + lr;
                if (row < g.M && col < g.N) {
                    if (g.nchunk > 1) {
                        g.P[((long long)chunk * g.M + row) * g.N + col] = acc[i][j][r];
                    } else {
                        double* c = g.C + row * g.ldc + col;
                        const double v = g.alpha * acc[i][j][r];
                        *c = (g.beta == 0.0) ? v : v + g.beta * (*c);
                    }
                }
            }
}

// ---------------------------------------------------------------------------
// The same product with Z given k-major (Zt[k][m], as G is [k][n]).  Both tiles then are
// plain row copies, so they go from HBM straight into LDS by buffer loads (16 bytes a lane,
// no registers, no stash): one load per tile row and wave, addressed by a per-lane offset
// fixed for the kernel and a per-slab scalar offset.  The buffer descriptors cover the
// chunk's rows only, so rows past the chunk's end read as zero and need no masking; columns
// past M or N may read neighbouring data, which only reaches output rows or columns that are
// never written.  The two LDS buffers are separate arrays so that the compiler can tell the
// loads into one from the reads of the other and waits for the loads only at the barrier.
// Byte offsets within a chunk are 32-bit: the host keeps each chunk below 2^31 bytes.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void* lds_ptr;

__device__ inline __amdgpu_buffer_rsrc_t chunk_rsrc(const double* base, long long bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000);
}

__device__ inline void block_tile(int nchunk, int ntn, int& chunk, int& nt) {
    const int b = blockIdx.x;
    if ((nchunk & 7) == 0) {
        const int q = b >> 3;
        chunk = (q / ntn) * 8 + (b & 7);
        nt = q % ntn;
    } else {
        chunk = b / ntn;
        nt = b % ntn;
    }
}

template <int TM, int TAG>
__global__ __launch_bounds__(LNT, 2) void ladder_f64t_kernel(LadderArgs g) {
    constexpr int BM = 16 * TM, RA = BM + 2, RB = LBN + 2;  // LDS row strides (doubles)
    __shared__ __attribute__((aligned(16))) double As0[LBK][RA], As1[LBK][RA];
    __shared__ __attribute__((aligned(16))) double Bs0[LBK][RB], Bs1[LBK][RB];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int chunk, nt;
    block_tile(g.nchunk, g.ntn, chunk, nt);
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)nt * LBN;
    const int kb = chunk * g.Kc, ke = min(g.K, kb + g.Kc);
    const __amdgpu_buffer_rsrc_t ra = chunk_rsrc(g.Z + (long long)kb * g.ldz + m0, (long long)(ke - kb) * g.ldz * 8 - m0 * 8);
    const __amdgpu_buffer_rsrc_t rb = chunk_rsrc(g.G + (long long)kb * g.ldg + n0, (long long)(ke - kb) * g.ldg * 8 - n0 * 8);
    // wave w copies rows 4w .. 4w+3 of both tiles; lane l the two elements at column 2l
    const bool acol = 2 * lane < BM;
    unsigned voa[4], vob[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        voa[r] = (unsigned)(((4 * wave + r) * g.ldz + 2 * lane) * 8);
        vob[r] = (unsigned)(((4 * wave + r) * g.ldg + 2 * lane) * 8);
    }
    auto issue = [&](double(&At)[LBK][RA], double(&Bt)[LBK][RB], int s) {
        const int soa = s * LBK * (int)g.ldz * 8, sob = s * LBK * (int)g.ldg * 8;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (acol) __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)&At[4 * wave + r][0], 16, voa[r], soa, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr)&Bt[4 * wave + r][0], 16, vob[r], sob, 0, 0);
        }
    };
    d4v acc[TM][LTN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j) acc[i][j] = d4v{0.0, 0.0, 0.0, 0.0};
    const int cb = wave * (16 * LTN);
    // Rows and columns are dealt to the MFMA blocks in interleaved pairs, so that one 16-byte LDS read
    // fetches the fragments of two blocks: row block 2h+e holds rows 32h + 2t + e, column block j holds
    // columns cb + 2t + j (t the fragment index, e and j 0 or 1); an odd TM reads its last row block
    // (rows 16(TM-1) + t) singly.  The epilogue maps the blocks back.
    auto compute = [&](const double(&At)[LBK][RA], const double(&Bt)[LBK][RB]) {
#pragma unroll
        for (int kk = 0; kk < LBK; kk += 4) {
            const d2v bq = *(const d2v*)&Bt[kk + lk][cb + 2 * lr];
#pragma unroll
            for (int h = 0; h < TM / 2; ++h) {
                const d2v aq = *(const d2v*)&At[kk + lk][32 * h + 2 * lr];
                acc[2 * h][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.x, bq.x, acc[2 * h][0], 0, 0, 0);
                acc[2 * h][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.x, bq.y, acc[2 * h][1], 0, 0, 0);
                acc[2 * h + 1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.y, bq.x, acc[2 * h + 1][0], 0, 0, 0);
                acc[2 * h + 1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq.y, bq.y, acc[2 * h + 1][1], 0, 0, 0);
            }
            if constexpr (TM & 1) {
                const double af = At[kk + lk][16 * (TM - 1) + lr];
                acc[TM - 1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bq.x, acc[TM - 1][0], 0, 0, 0);
                acc[TM - 1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bq.y, acc[TM - 1][1], 0, 0, 0);
            }
        }
    };
    // all of this wave's loads have landed in LDS (and its LDS reads are done), then the barrier
    auto sync = [] {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };
    const int nslab = (ke - kb + LBK - 1) / LBK;
    issue(As0, Bs0, 0);
    sync();
    int s = 0;
    for (; s + 1 < nslab; s += 2) {
        issue(As1, Bs1, s + 1);
        compute(As0, Bs0);
        sync();
        if (s + 2 < nslab) issue(As0, Bs0, s + 2);
        compute(As1, Bs1);
        sync();
    }
    if (s < nslab) compute(As0, Bs0);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = lk + 4 * r;  // the block's output row
                const long long row = m0 + ((TM & 1) && i == TM - 1 ? 16 * i + t : 32 * (i >> 1) + 2 * t + (i & 1));
                const long long col = n0 + cb + 2 * lr + j;
                if (row < g.M && col < g.N) {
                    if (g.nchunk > 1) {
                        g.P[((long long)chunk * g.M + row) * g.N + col] = acc[i][j][r];
                    } else {
                        double* c = g.C + row * g.ldc + col;
                        const double v = g.alpha * acc[i][j][r];
                        *c = (g.beta == 0.0) ? v : v + g.beta * (*c);
                    }
                }
            }
}

// ---------------------------------------------------------------------------
// Reduced-precision ladders (FP32 accumulation, FP64 partial sums / output).
//   FP32: v_mfma_f32_16x16x4f32, Z32[m][k] and G32[k][n] staged through LDS (BK 32).
//   BF16: v_mfma_f32_16x16x32_bf16.  G is symmetric, so column n of the B operand is
//         row n of G: each lane loads its 8 consecutive k straight from HBM into
//         registers (one slab ahead), and only the Z slab (shared by the 4 waves) goes
//         through LDS.  This kernel is bound by the G stream (2 bytes per element).
// FP32-output accumulator layout of both: element r holds D[4(l/16) + r][l%16].
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

struct LadderLP {
    const void* Z; long long ldz;
    const void* G; long long ldg;
    double* C; long long ldc;
    double* P;
    int M, N, K, Kc, ntn, nchunk;
    double alpha, beta;
};

template <int TM>
__device__ inline void store_f32_tile(const LadderLP& g, f4v (&acc)[TM][LTN], long long m0, long long n0, int cb,
                                      int chunk, int lr, int lk) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = m0 + 16 * i + 4 * lk + r;
                const long long col = n0 + cb + 16 * j + lr;
                if (row < g.M && col < g.N) {
                    if (g.nchunk > 1) {
                        g.P[((long long)chunk * g.M + row) * g.N + col] = (double)acc[i][j][r];
                    } else {
                        double* c = g.C + row * g.ldc + col;
                        const double v = g.alpha * (double)acc[i][j][r];
                        *c = (g.beta == 0.0) ? v : v + g.beta * (*c);
                    }
                }
            }
}

constexpr int FBK = 32;
template <int TM, int TAG>
__global__ __launch_bounds__(LNT, 2) void ladder_f32_kernel(LadderLP g) {
    constexpr int BM = 16 * TM;
    constexpr int PA = (BM * (FBK / 4) + LNT - 1) / LNT;
    constexpr int PB = (FBK * (LBN / 4)) / LNT;
    __shared__ __attribute__((aligned(16))) float As[2][FBK][BM + 1];  // transposed: [k][m]
    __shared__ __attribute__((aligned(16))) float Bs[2][FBK][LBN + 4];
    const float* __restrict__ Z = (const float*)g.Z;
    const float* __restrict__ G = (const float*)g.G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int chunk, nt;
    block_tile(g.nchunk, g.ntn, chunk, nt);
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)nt * LBN;
    const int kb = chunk * g.Kc, ke = min(g.K, kb + g.Kc);
    int arow[PA], akq[PA], bkr[PB], bnq[PB];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
        const int idx = tid + LNT * p;
        arow[p] = idx < BM * (FBK / 4) ? idx / (FBK / 4) : -1;
        akq[p] = idx % (FBK / 4);
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int idx = tid + LNT * p;
        bkr[p] = idx / (LBN / 4);
        bnq[p] = idx % (LBN / 4);
    }
    f4v ra[PA], rb[PB];
    const f4v z4 = {0.f, 0.f, 0.f, 0.f};
    auto fetch = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const long long m = m0 + arow[p];
            const int k = k0 + 4 * akq[p];
            ra[p] = (arow[p] >= 0 && m < g.M && k < ke) ? *(const f4v*)(Z + m * g.ldz + k) : z4;
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            const int k = k0 + bkr[p];
            const long long n = n0 + 4 * bnq[p];
            rb[p] = (k < ke && n < g.N) ? *(const f4v*)(G + (long long)k * g.ldg + n) : z4;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (arow[p] >= 0) {
#pragma unroll
                for (int q = 0; q < 4; ++q) As[buf][4 * akq[p] + q][arow[p]] = ra[p][q];
            }
#pragma unroll
        for (int p = 0; p < PB; ++p) *(f4v*)&Bs[buf][bkr[p]][4 * bnq[p]] = rb[p];
    };
    f4v acc[TM][LTN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j) acc[i][j] = z4;
    const int nslab = (ke - kb + FBK - 1) / FBK;
    if (nslab > 0) {
        fetch(kb);
        stash(0);
    }
    __syncthreads();
    const int cb = wave * (16 * LTN);
    for (int s = 0; s < nslab; ++s) {
        const int buf = s & 1;
        if (s + 1 < nslab) fetch(kb + (s + 1) * FBK);
#pragma unroll
        for (int kk = 0; kk < FBK; kk += 4) {
            float bf[LTN];
#pragma unroll
            for (int j = 0; j < LTN; ++j) bf[j] = Bs[buf][kk + lk][cb + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const float af = As[buf][kk + lk][16 * i + lr];
#pragma unroll
                for (int j = 0; j < LTN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf[j], acc[i][j], 0, 0, 0);
            }
        }
        if (s + 1 < nslab) stash(buf ^ 1);
        __syncthreads();
    }
    store_f32_tile<TM>(g, acc, m0, n0, cb, chunk, lr, lk);
}

// FP32 with Z k-major, both tiles copied HBM -> LDS by buffer loads as in ladder_f64t_kernel.  A
// tile row of 128 floats is 512 bytes, so each copy instruction moves one row on half the lanes,
// which lets every LDS row keep its padding.  32-deep slabs, two LDS buffers (separate arrays).
constexpr int FTK = 32;
template <int TM, int TAG>
__global__ __launch_bounds__(LNT, 2) void ladder_f32t_kernel(LadderLP g) {
    constexpr int BM = 16 * TM, RA = BM + 4, RB = LBN + 4;  // LDS row strides (floats)
    __shared__ __attribute__((aligned(16))) float As0[FTK][RA], As1[FTK][RA];
    __shared__ __attribute__((aligned(16))) float Bs0[FTK][RB], Bs1[FTK][RB];
    const float* __restrict__ Z = (const float*)g.Z;
    const float* __restrict__ G = (const float*)g.G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int chunk, nt;
    block_tile(g.nchunk, g.ntn, chunk, nt);
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)nt * LBN;
    const int kb = chunk * g.Kc, ke = min(g.K, kb + g.Kc);
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(Z + (long long)kb * g.ldz + m0), (short)0, (int)((long long)(ke - kb) * g.ldz * 4 - m0 * 4), 0x00020000);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(G + (long long)kb * g.ldg + n0), (short)0, (int)((long long)(ke - kb) * g.ldg * 4 - n0 * 4), 0x00020000);
    // wave w copies rows 8w .. 8w+7 of both tiles; lane l < 32 the four elements at column 4l
    const bool bcol = lane < 32, acol = 4 * lane < BM;
    unsigned voa[8], vob[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        voa[r] = (unsigned)(((8 * wave + r) * g.ldz + 4 * lane) * 4);
        vob[r] = (unsigned)(((8 * wave + r) * g.ldg + 4 * lane) * 4);
    }
    auto issue = [&](float(&At)[FTK][RA], float(&Bt)[FTK][RB], int s) {
        const int soa = s * FTK * (int)g.ldz * 4, sob = s * FTK * (int)g.ldg * 4;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (acol) __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)&At[8 * wave + r][0], 16, voa[r], soa, 0, 0);
            if (bcol) __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr)&Bt[8 * wave + r][0], 16, vob[r], sob, 0, 0);
        }
    };
    f4v acc[TM][LTN];
    const f4v z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j) acc[i][j] = z4;
    const int cb = wave * (16 * LTN);
    auto compute = [&](const float(&At)[FTK][RA], const float(&Bt)[FTK][RB]) {
#pragma unroll
        for (int kk = 0; kk < FTK; kk += 4) {
            float bf[LTN];
#pragma unroll
            for (int j = 0; j < LTN; ++j) bf[j] = Bt[kk + lk][cb + 16 * j + lr];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const float af = At[kk + lk][16 * i + lr];
#pragma unroll
                for (int j = 0; j < LTN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf[j], acc[i][j], 0, 0, 0);
            }
        }
    };
    auto sync = [] {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };
    const int nslab = (ke - kb + FTK - 1) / FTK;
    issue(As0, Bs0, 0);
    sync();
    int s = 0;
    for (; s + 1 < nslab; s += 2) {
        issue(As1, Bs1, s + 1);
        compute(As0, Bs0);
        sync();
        if (s + 2 < nslab) issue(As0, Bs0, s + 2);
        compute(As1, Bs1);
        sync();
    }
    if (s < nslab) compute(As0, Bs0);
    store_f32_tile<TM>(g, acc, m0, n0, cb, chunk, lr, lk);
}

constexpr int HBK = 64, HPAD = 8;
template <int TM, int TAG>
__global__ __launch_bounds__(LNT, 2) void ladder_bf16_kernel(LadderLP g) {
    constexpr int BM = 16 * TM;
    constexpr int PA = (BM * (HBK / 8) + LNT - 1) / LNT;
    __shared__ __attribute__((aligned(16))) __bf16 As[2][BM][HBK + HPAD];
    const __bf16* __restrict__ Z = (const __bf16*)g.Z;
    const __bf16* __restrict__ G = (const __bf16*)g.G;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    int chunk, nt;
    block_tile(g.nchunk, g.ntn, chunk, nt);
    const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)nt * LBN;
    const int kb = chunk * g.Kc, ke = min(g.K, kb + g.Kc);
    const int cb = wave * (16 * LTN);
    int arow[PA], akq[PA];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
        const int idx = tid + LNT * p;
        arow[p] = idx < BM * (HBK / 8) ? idx / (HBK / 8) : -1;
        akq[p] = idx % (HBK / 8);
    }
    bf8v ra[PA], rb[LTN][2];
    bf8v zero8;
#pragma unroll
    for (int q = 0; q < 8; ++q) zero8[q] = (__bf16)0.f;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const long long m = m0 + arow[p];
            const int k = k0 + 8 * akq[p];
            ra[p] = (arow[p] >= 0 && m < g.M && k < ke) ? *(const bf8v*)(Z + m * g.ldz + k) : zero8;
        }
#pragma unroll
        for (int j = 0; j < LTN; ++j) {
            const long long col = n0 + cb + 16 * j + lr;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int k = k0 + 32 * ks + 8 * lk;
                rb[j][ks] = (col < g.N && k < ke) ? *(const bf8v*)(G + col * g.ldg + k) : zero8;
            }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (arow[p] >= 0) *(bf8v*)&As[buf][arow[p]][8 * akq[p]] = ra[p];
    };
    f4v acc[TM][LTN];
    const f4v z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < LTN; ++j) acc[i][j] = z4;
    const int nslab = (ke - kb + HBK - 1) / HBK;
    bf8v cbf[LTN][2];
    if (nslab > 0) {
        fetch(kb);
        stash(0);
    }
    __syncthreads();
    for (int s = 0; s < nslab; ++s) {
        const int buf = s & 1;
#pragma unroll
        for (int j = 0; j < LTN; ++j)
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) cbf[j][ks] = rb[j][ks];
        if (s + 1 < nslab) fetch(kb + (s + 1) * HBK);
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int i = 0; i < TM; ++i) {
                const bf8v af = *(const bf8v*)&As[buf][16 * i + lr][32 * ks + 8 * lk];
#pragma unroll
                for (int j = 0; j < LTN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, cbf[j][ks], acc[i][j], 0, 0, 0);
            }
        if (s + 1 < nslab) stash(buf ^ 1);
        __syncthreads();
    }
    store_f32_tile<TM>(g, acc, m0, n0, cb, chunk, lr, lk);
}

template <int TM, int TAG>
void launch_lp_tm(const LadderLP& a, int prec, int mtiles, hipStream_t s) {
    if (prec == 1) hipLaunchKernelGGL((ladder_f32_kernel<TM, TAG>), dim3(a.nchunk * a.ntn, mtiles), dim3(LNT), 0, s, a);
    else hipLaunchKernelGGL((ladder_bf16_kernel<TM, TAG>), dim3(a.nchunk * a.ntn, mtiles), dim3(LNT), 0, s, a);
}

template <int TAG>
void launch_lp_tag(const LadderLP& a, int prec, int tm, int mtiles, hipStream_t s) {
    switch (tm) {
        case 1: launch_lp_tm<1, TAG>(a, prec, mtiles, s); break;
        case 2: launch_lp_tm<2, TAG>(a, prec, mtiles, s); break;
        case 3: launch_lp_tm<3, TAG>(a, prec, mtiles, s); break;
        case 4: launch_lp_tm<4, TAG>(a, prec, mtiles, s); break;
        case 5: launch_lp_tm<5, TAG>(a, prec, mtiles, s); break;
        case 6: launch_lp_tm<6, TAG>(a, prec, mtiles, s); break;
        case 7: launch_lp_tm<7, TAG>(a, prec, mtiles, s); break;
        default: launch_lp_tm<8, TAG>(a, prec, mtiles, s); break;
    }
}

template <int TM, int TAG>
void launch_f32t_tm(const LadderLP& a, int mtiles, hipStream_t s) {
    hipLaunchKernelGGL((ladder_f32t_kernel<TM, TAG>), dim3(a.nchunk * a.ntn, mtiles), dim3(LNT), 0, s, a);
}

template <int TAG>
void launch_f32t_tag(const LadderLP& a, int tm, int mtiles, hipStream_t s) {
    switch (tm) {
        case 1: launch_f32t_tm<1, TAG>(a, mtiles, s); break;
        case 2: launch_f32t_tm<2, TAG>(a, mtiles, s); break;
        case 3: launch_f32t_tm<3, TAG>(a, mtiles, s); break;
        case 4: launch_f32t_tm<4, TAG>(a, mtiles, s); break;
        case 5: launch_f32t_tm<5, TAG>(a, mtiles, s); break;
        case 6: launch_f32t_tm<6, TAG>(a, mtiles, s); break;
        case 7: launch_f32t_tm<7, TAG>(a, mtiles, s); break;
        default: launch_f32t_tm<8, TAG>(a, mtiles, s); break;
    }
}

void launch_lp(const LadderLP& a, int prec, int tm, int mtiles, bool trial, hipStream_t s) {
    if (trial) launch_lp_tag<1>(a, prec, tm, mtiles, s);
    else launch_lp_tag<0>(a, prec, tm, mtiles, s);
    LAUNCHCHK();
}

template <int TM, int TAG>
void launch_tm(const LadderArgs& a, int mtiles, hipStream_t s) {
    hipLaunchKernelGGL((ladder_f64_kernel<TM, TAG>), dim3(a.nchunk * a.ntn, mtiles), dim3(LNT), 0, s, a);
}

template <int TAG>
void launch_tag(const LadderArgs& a, int tm, int mtiles, hipStream_t s) {
    switch (tm) {
        case 1: launch_tm<1, TAG>(a, mtiles, s); break;
        case 2: launch_tm<2, TAG>(a, mtiles, s); break;
        case 3: launch_tm<3, TAG>(a, mtiles, s); break;
        case 4: launch_tm<4, TAG>(a, mtiles, s); break;
        case 5: launch_tm<5, TAG>(a, mtiles, s); break;
        case 6: launch_tm<6, TAG>(a, mtiles, s); break;
        case 7: launch_tm<7, TAG>(a, mtiles, s); break;
        default: launch_tm<8, TAG>(a, mtiles, s); break;
    }
}

void launch(const LadderArgs& a, int tm, int mtiles, int tag, hipStream_t s) {
    if (tag == 1) launch_tag<1>(a, tm, mtiles, s);
    else if (tag == 2) launch_tag<2>(a, tm, mtiles, s);
    else launch_tag<0>(a, tm, mtiles, s);
    LAUNCHCHK();
}

template <int TM, int TAG>
void launch_t_tm(const LadderArgs& a, int mtiles, hipStream_t s) {
    hipLaunchKernelGGL((ladder_f64t_kernel<TM, TAG>), dim3(a.nchunk * a.ntn, mtiles), dim3(LNT), 0, s, a);
}

template <int TAG>
void launch_t_tag(const LadderArgs& a, int tm, int mtiles, hipStream_t s) {
    switch (tm) {
        case 1: launch_t_tm<1, TAG>(a, mtiles, s); break;
        case 2: launch_t_tm<2, TAG>(a, mtiles, s); break;
        case 3: launch_t_tm<3, TAG>(a, mtiles, s); break;
        case 4: launch_t_tm<4, TAG>(a, mtiles, s); break;
        case 5: launch_t_tm<5, TAG>(a, mtiles, s); break;
        case 6: launch_t_tm<6, TAG>(a, mtiles, s); break;
        case 7: launch_t_tm<7, TAG>(a, mtiles, s); break;
        default: launch_t_tm<8, TAG>(a, mtiles, s); break;
    }
}
}  // namespace

// Row tiling: as few tiles of <= 128 rows as possible (each tile streams G once), each
// as short as those rows allow (padding rows cost matrix-core time).
void ladder_rows(int M, int& tm, int& mtiles) {
    mtiles = (M + 127) / 128;
    tm = (M + 16 * mtiles - 1) / (16 * mtiles);
}

namespace {
thread_local int t_trial_rows = 0;  // row-tile count of a tuner trial launch (0: none)
}
static int tuned_rows(int prec, int M, int N, int K);

// The row tiling a launch uses: the tuner's measured choice for the shape (more, shorter tiles: G
// streamed once per tile, more workgroups) where it has one, else the default above.
static void rows_for(int prec, int M, int N, int K, int& tm, int& mtiles) {
    ladder_rows(M, tm, mtiles);
    const int mt = t_trial_rows > 0 ? t_trial_rows : tuned_rows(prec, M, N, K);
    if (mt > mtiles) {
        const int t = (M + 16 * mt - 1) / (16 * mt);
        if (t >= 1 && t <= 8) {
            tm = t;
            mtiles = mt;
        }
    }
}

bool ladder_supported(int M, int N, int K, const double* Z, long long ldz, const double* G, long long ldg,
                      const double* C, long long ldc) {
    auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    return M > 0 && N > 0 && K > 0 && (N % 2 == 0) && (K % 2 == 0) && (ldz % 2 == 0) && (ldg % 2 == 0) &&
           (ldc % 2 == 0) && al16(Z) && al16(G) && al16(C);
}

// K per chunk: a multiple of the slab depth of every ladder kernel (64)
int ladder_chunk_len(int K, int nchunk) {
    const int kc = (K + nchunk - 1) / nchunk;
    return (kc + 63) / 64 * 64;
}

bool ladder_lp_supported(int prec, int M, int N, int K, const void* Z, long long ldz, const void* G, long long ldg,
                         const double* C, long long ldc) {
    auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    if (!(M > 0 && N > 0 && K > 0 && al16(Z) && al16(G) && al16(C) && ldc % 2 == 0)) return false;
    if (prec == 1) return N % 4 == 0 && K % 4 == 0 && ldz % 4 == 0 && ldg % 4 == 0;
    if (prec == 2) return N == K && K % 8 == 0 && ldz % 8 == 0 && ldg % 8 == 0;  // B read through symmetry
    return false;
}

void ladder_gemm_lp(int prec, int M, int N, int K, double alpha, const void* Z, long long ldz, const void* G,
                    long long ldg, double beta, double* C, long long ldc, int nchunk, double* partial,
                    long long partial_elems, hipStream_t s, bool trial) {
    if (g_dry || M <= 0 || N <= 0) return;
    int tm, mtiles;
    rows_for(prec, M, N, K, tm, mtiles);
    nchunk = std::max(1, std::min(nchunk, (K + 255) / 256));
    if (nchunk > 1 && (!partial || (long long)nchunk * M * N > partial_elems)) nchunk = 1;
    LadderLP a;
    a.Z = Z; a.ldz = ldz; a.G = G; a.ldg = ldg; a.C = C; a.ldc = ldc; a.P = partial;
    a.M = M; a.N = N; a.K = K;
    a.Kc = ladder_chunk_len(K, nchunk);
    a.nchunk = (K + a.Kc - 1) / a.Kc;
    a.ntn = (N + LBN - 1) / LBN;
    a.alpha = alpha; a.beta = beta;
    launch_lp(a, prec, tm, mtiles, trial, s);
    if (a.nchunk > 1) splitk_reduce(partial, a.nchunk, M, N, alpha, beta, C, ldc, 1, s);
}

void ladder_gemm(int M, int N, int K, double alpha, const double* Z, long long ldz, const double* G, long long ldg,
                 double beta, double* C, long long ldc, int nchunk, double* partial, long long partial_elems,
                 hipStream_t s, int tag) {
    if (g_dry || M <= 0 || N <= 0) return;
    int tm, mtiles;
    rows_for(0, M, N, K, tm, mtiles);
    nchunk = std::max(1, std::min(nchunk, (K + 255) / 256));
    if (nchunk > 1 && (!partial || (long long)nchunk * M * N > partial_elems)) nchunk = 1;
    LadderArgs a;
    a.Z = Z; a.ldz = ldz; a.G = G; a.ldg = ldg; a.C = C; a.ldc = ldc; a.P = partial;
    a.M = M; a.N = N; a.K = K;
    a.Kc = ladder_chunk_len(K, nchunk);
    a.nchunk = (K + a.Kc - 1) / a.Kc;
    a.ntn = (N + LBN - 1) / LBN;
    a.alpha = alpha; a.beta = beta;
    launch(a, tm, mtiles, tag, s);
    if (a.nchunk > 1) splitk_reduce(partial, a.nchunk, M, N, alpha, beta, C, ldc, 1, s);
}

// ---------------------------------------------------------------------------
// Autotuner for the chunk count.  The best split depends on M (rows per tile), the
// column count and the chip's load balance, so it is measured: on the first call for a
// (rows, N, K) shape each candidate (chunk count, and row tiling where that matters) runs once
// untimed, then in three interleaved rounds timed launch by launch with HIP events on the
// caller's stream; the candidate with the fastest single launch is kept for the process.  One
// shape is measured at a time, other threads that reach it wait for the result, and taking each
// candidate's best round keeps other streams' kernels from deciding it.  ADC3_TUNE_CACHE names a
// text file that keeps the choices across processes (one line per shape and device
// architecture); ADC3_LADDER_CHUNKS fixes the count and disables tuning.  Different
// chunk counts sum in a different order, so the last bits of sigma can differ between
// choices, never between two calls that use the same choice.
// ---------------------------------------------------------------------------
// Chunks of the k-major kernel are addressed with 32-bit byte offsets: the smallest chunk count
// whose chunks (a multiple of 64 rows each) stay below 2^31 bytes in both operands, or 0 when
// not even 64 rows fit.
// (adc3_debug_ladder_offset_limit lowers the byte limit for tests of the multi-chunk paths)
static std::atomic<long long> g_offset_limit{0};
static long long offset_limit() {
    const long long l = g_offset_limit.load();
    return l > 0 ? l : (1LL << 31) - 1;
}
int ladder_t_min_chunks(int K, long long ldz, long long ldg) {
    const long long ld = std::max(ldz, ldg);
    if (K <= 0 || ld <= 0) return 0;
    const long long kcmax = offset_limit() / (8 * ld) / 64 * 64;
    if (kcmax < 64) return 0;
    int n = (int)std::max<long long>(1, (K + kcmax - 1) / kcmax);
    while (ladder_chunk_len(K, n) > kcmax) ++n;
    return n;
}

bool ladder_t_supported(int M, int N, int K, const double* Zt, long long ldz, const double* G, long long ldg) {
    auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    return M > 0 && N > 0 && K > 0 && ldz >= M && ldg >= N && ldz % 2 == 0 && ldg % 2 == 0 && al16(Zt) && al16(G) &&
           ladder_t_min_chunks(K, ldz, ldg) > 0;
}

bool ladder_gemm_t(int M, int N, int K, double alpha, const double* Zt, long long ldz, const double* G, long long ldg,
                   double beta, double* C, long long ldc, int nchunk, double* partial, long long partial_elems,
                   hipStream_t s, int tag) {
    if (M <= 0 || N <= 0) return true;
    const int nmin = ladder_t_min_chunks(K, ldz, ldg);
    if (nmin <= 0) return false;
    nchunk = std::max(nmin, std::min(nchunk, (K + 255) / 256));
    if (nchunk > 1 && (!partial || (long long)nchunk * M * N > partial_elems)) return false;
    if (g_dry) return true;
    int tm, mtiles;
    rows_for(3, M, N, K, tm, mtiles);
    LadderArgs a;
    a.Z = Zt; a.ldz = ldz; a.G = G; a.ldg = ldg; a.C = C; a.ldc = ldc; a.P = partial;
    a.M = M; a.N = N; a.K = K;
    a.Kc = ladder_chunk_len(K, nchunk);
    a.nchunk = (K + a.Kc - 1) / a.Kc;
    a.ntn = (N + LBN - 1) / LBN;
    a.alpha = alpha; a.beta = beta;
    if (tag == 1) launch_t_tag<1>(a, tm, mtiles, s);
    else if (tag == 2) launch_t_tag<2>(a, tm, mtiles, s);
    else launch_t_tag<0>(a, tm, mtiles, s);
    LAUNCHCHK();
    if (a.nchunk > 1) splitk_reduce(partial, a.nchunk, M, N, alpha, beta, C, ldc, 1, s);
    return true;
}

int ladder_t32_min_chunks(int K, long long ldz, long long ldg) {
    const long long ld = std::max(ldz, ldg);
    if (K <= 0 || ld <= 0) return 0;
    const long long kcmax = ((1LL << 31) - 1) / (4 * ld) / 64 * 64;
    if (kcmax < 64) return 0;
    int n = (int)std::max<long long>(1, (K + kcmax - 1) / kcmax);
    while (ladder_chunk_len(K, n) > kcmax) ++n;
    return n;
}

bool ladder_t32_supported(int M, int N, int K, const float* Zt, long long ldz, const float* G, long long ldg) {
    auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    return M > 0 && N > 0 && K > 0 && ldz >= M && ldg >= N && ldz % 4 == 0 && ldg % 4 == 0 && al16(Zt) && al16(G) &&
           ladder_t32_min_chunks(K, ldz, ldg) > 0;
}

bool ladder_gemm_t32(int M, int N, int K, double alpha, const float* Zt, long long ldz, const float* G, long long ldg,
                     double beta, double* C, long long ldc, int nchunk, double* partial, long long partial_elems,
                     hipStream_t s, int tag) {
    if (M <= 0 || N <= 0) return true;
    const int nmin = ladder_t32_min_chunks(K, ldz, ldg);
    if (nmin <= 0) return false;
    nchunk = std::max(nmin, std::min(nchunk, (K + 255) / 256));
    if (nchunk > 1 && (!partial || (long long)nchunk * M * N > partial_elems)) return false;
    if (g_dry) return true;
    int tm, mtiles;
    rows_for(4, M, N, K, tm, mtiles);
    LadderLP a;
    a.Z = Zt; a.ldz = ldz; a.G = G; a.ldg = ldg; a.C = C; a.ldc = ldc; a.P = partial;
    a.M = M; a.N = N; a.K = K;
    a.Kc = ladder_chunk_len(K, nchunk);
    a.nchunk = (K + a.Kc - 1) / a.Kc;
    a.ntn = (N + LBN - 1) / LBN;
    a.alpha = alpha; a.beta = beta;
    if (tag == 1) launch_f32t_tag<1>(a, tm, mtiles, s);
    else launch_f32t_tag<0>(a, tm, mtiles, s);
    LAUNCHCHK();
    if (a.nchunk > 1) splitk_reduce(partial, a.nchunk, M, N, alpha, beta, C, ldc, 1, s);
    return true;
}

namespace {
std::mutex g_tune_mu;
std::mutex g_tune_run_mu;  // held while a shape's trial launches run: one shape measured at a time
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

// architecture name of the current device, looked up once per device (the key of tuned shapes)
std::string arch_name() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
    std::string a = pr.gcnArchName;
    a = a.substr(0, a.find(':'));
    names[dev] = a;
    return a;
}

std::string tune_key(int prec, int M, int N, int K) {
    int tm, mt;
    ladder_rows(M, tm, mt);
    return std::string(prec == 0 ? "ladder_f64 " : prec == 1 ? "ladder_f32 " : prec == 2 ? "ladder_bf16 " : prec == 3 ? "ladder_f64t " : "ladder_f32t ") + arch_name() + " " + std::to_string(tm) + " " + std::to_string(mt) + " " +
           std::to_string(N) + " " + std::to_string(K);
}

void load_cache() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("ADC3_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        const size_t sp = l.find_last_of(' ');
        if (sp == std::string::npos) continue;
        const int v = std::atoi(l.c_str() + sp + 1);
        if (v >= 1) g_tune[l.substr(0, sp)] = v;
    }
    std::fclose(f);
}

std::string rows_key(const std::string& key) { return key + " rows"; }

void store_cache(const std::string& key, int v) {
    const char* path = std::getenv("ADC3_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d\n", key.c_str(), v);
    std::fclose(f);
}
}  // namespace

static int tuned_rows(int prec, int M, int N, int K) {
    if (g_dry) return 0;
    const std::string key = rows_key(tune_key(prec, M, N, K));
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache();
    auto it = g_tune.find(key);
    return it == g_tune.end() ? 0 : it->second;
}

static void ladder_run(int prec, int M, int N, int K, const void* Z, long long ldz, const void* G, long long ldg,
                       double* C, long long ldc, int nchunk, double* partial, long long pe, hipStream_t s) {
    if (prec == 0)
        ladder_gemm(M, N, K, 1.0, (const double*)Z, ldz, (const double*)G, ldg, 0.0, C, ldc, nchunk, partial, pe, s,
                    1);
    else if (prec == 3)
        ladder_gemm_t(M, N, K, 1.0, (const double*)Z, ldz, (const double*)G, ldg, 0.0, C, ldc, nchunk, partial, pe, s, 1);
    else if (prec == 4)
        ladder_gemm_t32(M, N, K, 1.0, (const float*)Z, ldz, (const float*)G, ldg, 0.0, C, ldc, nchunk, partial, pe, s, 1);
    else
        ladder_gemm_lp(prec, M, N, K, 1.0, Z, ldz, G, ldg, 0.0, C, ldc, nchunk, partial, pe, s, true);
}

int ladder_tuned_chunks(int prec, int M, int N, int K, const void* Z, long long ldz, const void* G, long long ldg,
                        double* C, long long ldc, double* partial, long long partial_elems, hipStream_t s) {
    const char* fixed = std::getenv("ADC3_LADDER_CHUNKS");
    if (fixed && *fixed) return std::max(1, std::atoi(fixed));
    const int def = std::max(8, prec == 3 ? ladder_t_min_chunks(K, ldz, ldg) : prec == 4 ? ladder_t32_min_chunks(K, ldz, ldg) : 1);
    if (g_dry) return def;
    // a count tuned earlier for this shape holds under graph capture too (the eager pass before a
    // capture tunes it); only the trial launches themselves must stay out of a capture
    const std::string key = tune_key(prec, M, N, K);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_cache();
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) return def;
    // one shape measured at a time: host threads that reach the same shape together (the bases of a solve,
    // the instances of a batch) wait for the first one's result instead of timing it again
    std::unique_lock<std::mutex> run_lk(g_tune_run_mu);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) return it->second;
    }
    // prec 3 is the FP64 kernel with Z k-major, whose chunks have a minimum count
    const int nmin = prec == 3 ? ladder_t_min_chunks(K, ldz, ldg) : prec == 4 ? ladder_t32_min_chunks(K, ldz, ldg) : 1;
    std::vector<int> cand;
    for (int c : {1, 2, 4, 8, 16}) {
        if (c < nmin) continue;
        if (c > 1 && (long long)c * M * N > partial_elems) continue;
        if (c > 1 && K / c < 256) continue;
        cand.push_back(c);
    }
    if (cand.empty()) return std::max(nmin, 1);
    // row tilings: the default (fewest tiles), and one more, shorter tile (twice the workgroups for a
    // single tile, G streamed once more) where K chunks alone cannot give the chip 512 workgroups
    int tm0, mt0;
    ladder_rows(M, tm0, mt0);
    std::vector<int> rows{mt0};
    const long long ntn = (N + LBN - 1) / LBN;
    if (M > 16 * mt0 && ntn * mt0 * cand.back() < 512) rows.push_back(mt0 + 1);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // every (row tiling, chunk count) once untimed, then three rounds over all of them, each launch timed on
    // its own; a candidate's fastest round counts (kernels of other streams running beside a trial only
    // ever add time, and interleaving spreads them over the candidates)
    std::vector<std::pair<int, int>> trials;
    for (int mt : rows)
        for (int c : cand) trials.emplace_back(mt, c);
    std::vector<float> tbest(trials.size(), 1e30f);
    int best = cand[0], best_rows = mt0;
    try {
        for (const auto& t : trials) {
            t_trial_rows = t.first;
            ladder_run(prec, M, N, K, Z, ldz, G, ldg, C, ldc, t.second, partial, partial_elems, s);
        }
        for (int round = 0; round < 3; ++round)
            for (size_t i = 0; i < trials.size(); ++i) {
                t_trial_rows = trials[i].first;
                HIPCHK(hipEventRecord(e0, s));
                ladder_run(prec, M, N, K, Z, ldz, G, ldg, C, ldc, trials[i].second, partial, partial_elems, s);
                HIPCHK(hipEventRecord(e1, s));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                tbest[i] = std::min(tbest[i], ms);
            }
    } catch (...) {
        t_trial_rows = 0;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    size_t ib = 0;
    for (size_t i = 1; i < trials.size(); ++i)
        if (tbest[i] < tbest[ib]) ib = i;
    best_rows = trials[ib].first;
    best = trials[ib].second;
    t_trial_rows = 0;
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = best;
        g_tune[rows_key(key)] = best_rows;
        store_cache(key, best);
        store_cache(rows_key(key), best_rows);
    }
    return best;
}

}  // namespace adc3

extern "C" void adc3_debug_ladder_offset_limit(long long bytes) { adc3::g_offset_limit.store(bytes > 0 ? bytes : 0); }
