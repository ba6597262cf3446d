// The ladder term assembled from the DF factor, without the stored four-virtual matrix.
//
//   C_m = sum_Q B^Q Z_m B^Q,   i.e.  C_m[a][b] = sum_cd (ac|bd) Z_m[c][d],  (ac|bd) = sum_Q B^Q_ac B^Q_bd (eq 25)
//
// for rows m < M ((vector, occupied) pairs of a sigma pass, or (i,j) amplitude pairs), with
// B^Q = Bvv[Q] the symmetric v x v virtual block of the factor.  Per chunk of q auxiliary
// functions, two matrix-core contractions:
//   1. V[m][a][Qi][e] = sum_c B^Q[a][c] Z_m[c][e]              batched over (Qi, m): q*M products v x v x v
//   2. C[(m,a)][b]   += sum_(Qi,e) V[(m,a)][(Qi,e)] B^Q[e][b]  one GEMM with K = q*v
// 4 X M v^3 flops in all, against 2 M v^4 for the stored matrix: the cheaper form once X < v/2,
// and the only one once v^4 no longer fits in HBM (v = 600: 1 TB in FP64).
//
// FP64 and FP32 operands: one tile kernel serves both steps (16x16x4 MFMA, FP64 or FP32
// accumulation): 4 waves side by side over 128 columns, TM blocks of 16 rows, double-buffered
// LDS slabs, 16-byte loads where the shape allows (scalar loads otherwise), and two levels of
// batch offsets.  BF16 operands: both steps read their operands k-contiguous (Z transposed per row
// for step 1, the rows of B^Q itself for step 2, through its symmetry) and run on a kernel of
// their own (dfb_kernel, 32x32x16 MFMA, tiles copied HBM -> LDS by buffer loads); shapes it
// cannot take (v not a multiple of 8) fall back to the tile kernel with BF16 16x16x32 MFMA.
//
// MFMA layouts (lane l of a wave64):
//   f64 16x16x4 / f32 16x16x4: A frag A[l%16][l/16], B frag B[l/16][l%16]
//   bf16 16x16x32:             A frag A[l%16][8(l/16) .. +8], B frag B[8(l/16) .. +8][l%16]
//   bf16 32x32x16:             A frag A[l%32][8(l/32) .. +8], B frag B[8(l/32) .. +8][l%32]
//   accumulator element r: f64 row l/16 + 4r; FP32-output 16x16 instructions row 4(l/16) + r,
//   column l%16; 32x32x16 row 8(r/4) + 4(l/32) + r%4, column l%32.
#include "internal.h"
#include <algorithm>

namespace adc3 {

namespace {
typedef double d2x __attribute__((ext_vector_type(2)));
typedef double d4x __attribute__((ext_vector_type(4)));
typedef float f4x __attribute__((ext_vector_type(4)));
typedef __bf16 h8x __attribute__((ext_vector_type(8)));

constexpr int DNT = 256, DBN = 128, DLTN = 2;  // 4 waves x 2 column blocks of 16

struct DflArgs {
    const void* A; long long lda, bA0, bA1;  // A[m][k], row-major
    // B[k][n] row-major; with BT (BF16 only) B is read as Bt[n][k] at n*ldb + (k/kin)*ldbq + k%kin
    const void* B; long long ldb, bB0, bB1, ldbq;
    int kin;
    void* C; long long ldc, bC0, bC1;        // C[m][n]
    long long m_off;                         // first row of this launch
    int M, N, K, nb0;
    int accumulate;  // 1: C += A B, 0: C = A B
    int vec;         // 1: 16-byte loads (widths, strides and bases are multiples of the vector)
};

// per-precision element type, vector of 16 bytes, slab depth and accumulator
template <int P> struct Prec;
template <> struct Prec<0> { typedef double T; typedef d2x V; typedef d4x Acc; static constexpr int W = 2, BK = 16; };
template <> struct Prec<1> { typedef float T; typedef f4x V; typedef f4x Acc; static constexpr int W = 4, BK = 32; };
template <> struct Prec<2> { typedef __bf16 T; typedef h8x V; typedef f4x Acc; static constexpr int W = 8, BK = 64; };

template <int TO> struct Out;
template <> struct Out<0> { typedef double T; };
template <> struct Out<1> { typedef float T; };
template <> struct Out<2> { typedef __bf16 T; };

// VEC: 16-byte loads (K, the row strides, the batch offsets and, for B as [n][k], kin are multiples of
// the vector and the bases are 16-byte aligned); otherwise element loads with a bound on each element
template <int P, int TO, int TM, bool BT, bool VEC>
__global__ __launch_bounds__(DNT, 2) void dfl_kernel(DflArgs g) {
    static_assert(!BT || P == 2, "B given as [n][k] only for BF16");
    typedef typename Prec<P>::T T;
    typedef typename Prec<P>::V VT;
    typedef typename Prec<P>::Acc Acc;
    typedef typename Out<TO>::T OT;
    constexpr int W = Prec<P>::W, BK = Prec<P>::BK, BM = 16 * TM;
    constexpr int PA = (BM * (BK / W) + DNT - 1) / DNT;  // A vectors per thread and slab
    constexpr int PB = (BK * (DBN / W)) / DNT;             // B vectors per thread and slab
    // FP64/FP32: A transposed [k][m], B [k][n];  BF16: A [m][k], B transposed [n][k]
    constexpr int AR = (P == 2) ? BM : BK, AC = (P == 2) ? BK + 8 : BM + 1;
    constexpr int BR = (P == 2) ? DBN : BK, BC = (P == 2) ? BK + 8 : DBN + 16 / (int)sizeof(T);
    __shared__ __attribute__((aligned(16))) T As[2][AR][AC];
    __shared__ __attribute__((aligned(16))) T Bs[2][BR][BC];

    // Workgroup id H goes to XCD H % 8; give each XCD a contiguous range of the logical tile order
    // (column tiles fastest, then row tiles, then batches), so that the workgroups sharing a row strip
    // or a batch's operands run together under one L2
    int tx, ty, tz;
    {
        const unsigned long long gx = gridDim.x, gy = gridDim.y;
        const unsigned long long total = gx * gy * gridDim.z;
        const unsigned long long H = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
        const unsigned long long per = total / 8, rem = total % 8, x = H % 8, j = H / 8;
        const unsigned long long L = x * per + (x < rem ? x : rem) + j;
        tx = (int)(L % gx);
        ty = (int)((L / gx) % gy);
        tz = (int)(L / (gx * gy));
    }
    const int z = tz, b0 = z % g.nb0, b1 = z / g.nb0;
    const T* __restrict__ A = (const T*)g.A + b0 * g.bA0 + b1 * g.bA1;
    const T* __restrict__ B = (const T*)g.B + b0 * g.bB0 + b1 * g.bB1;
    OT* __restrict__ C = (OT*)g.C + b0 * g.bC0 + b1 * g.bC1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long long m0 = g.m_off + (long long)ty * BM, n0 = (long long)tx * DBN;
    const int K = g.K;

    int arow[PA], akq[PA], bkr[PB], bnq[PB];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
        const int idx = tid + DNT * p;
        arow[p] = idx < BM * (BK / W) ? idx / (BK / W) : -1;
        akq[p] = idx % (BK / W);
    }
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        const int idx = tid + DNT * p;
        if constexpr (BT) {  // bkr: column n, bnq: k vector
            bkr[p] = idx / (BK / W);
            bnq[p] = idx % (BK / W);
        } else {
            bkr[p] = idx / (DBN / W);
            bnq[p] = idx % (DBN / W);
        }
    }
    VT ra[PA], rb[PB];
    // per-thread row pointers, fixed for the whole K loop
    const T* ap[PA];
    bool aok[PA];
#pragma unroll
    for (int p = 0; p < PA; ++p) {
        const long long m = m0 + arow[p];
        aok[p] = arow[p] >= 0 && m < g.M;
        ap[p] = A + (aok[p] ? m * g.lda : 0) + W * akq[p];
    }
    const T* bp[PB];
    bool bok[PB];
#pragma unroll
    for (int p = 0; p < PB; ++p) {
        if constexpr (BT) {
            const long long n = n0 + bkr[p];
            bok[p] = n < g.N;
            bp[p] = B + (bok[p] ? n * g.ldb : 0);
        } else {
            const long long n = n0 + W * bnq[p];
            bok[p] = VEC ? n < g.N : true;
            bp[p] = B + (long long)bkr[p] * g.ldb + n;
        }
    }
    // B as [n][k]: k0 = kq * kin + kr, advanced by BK per slab without a division (kin >= BK)
    const bool kstep = g.kin >= BK;
    int kq = 0, kr = 0;
    auto fetch = [&](int k0) {
        const VT zv = {};
#pragma unroll
        for (int p = 0; p < PA; ++p) {
            const int k = k0 + W * akq[p];
            VT x = zv;
            if constexpr (VEC) {
                if (aok[p] && k < K) x = *(const VT*)(ap[p] + k0);
            } else {
                if (aok[p]) {
#pragma unroll
                    for (int e = 0; e < W; ++e)
                        if (k + e < K) x[e] = ap[p][k0 + e];
                }
            }
            ra[p] = x;
        }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            VT x = zv;
            if constexpr (BT) {
                const int k = k0 + W * bnq[p];
                if (bok[p]) {
                    if constexpr (VEC) {
                        if (k < K) {
                            long long off;
                            if (kstep) {
                                int r = kr + W * bnq[p], q = kq;
                                if (r >= g.kin) { r -= g.kin; ++q; }
                                off = (long long)q * g.ldbq + r;
                            } else {
                                off = (long long)(k / g.kin) * g.ldbq + k % g.kin;
                            }
                            x = *(const VT*)(bp[p] + off);
                        }
                    } else {
#pragma unroll
                        for (int e = 0; e < W; ++e)
                            if (k + e < K) x[e] = bp[p][(long long)((k + e) / g.kin) * g.ldbq + (k + e) % g.kin];
                    }
                }
            } else {
                const int k = k0 + bkr[p];
                if (k < K) {
                    const T* src = bp[p] + (long long)k0 * g.ldb;
                    if constexpr (VEC) {
                        if (bok[p]) x = *(const VT*)src;
                    } else {
                        const long long n = n0 + W * bnq[p];
#pragma unroll
                        for (int e = 0; e < W; ++e)
                            if (n + e < g.N) x[e] = src[e];
                    }
                }
            }
            rb[p] = x;
        }
        if (kstep) {
            kr += BK;
            if (kr >= g.kin) { kr -= g.kin; ++kq; }
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int p = 0; p < PA; ++p)
            if (arow[p] >= 0) {
                if constexpr (P == 2) {
                    *(VT*)&As[buf][arow[p]][W * akq[p]] = ra[p];
                } else {
#pragma unroll
                    for (int e = 0; e < W; ++e) As[buf][W * akq[p] + e][arow[p]] = ra[p][e];
                }
            }
#pragma unroll
        for (int p = 0; p < PB; ++p) {
            if constexpr (BT) {
                *(VT*)&Bs[buf][bkr[p]][W * bnq[p]] = rb[p];
            } else if constexpr (P == 2) {
#pragma unroll
                for (int e = 0; e < W; ++e) Bs[buf][W * bnq[p] + e][bkr[p]] = rb[p][e];
            } else {
                *(VT*)&Bs[buf][bkr[p]][W * bnq[p]] = rb[p];
            }
        }
    };

    Acc acc[TM][DLTN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < DLTN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;
    const int nslab = (K + BK - 1) / BK;
    if (nslab > 0) {
        fetch(0);
        stash(0);
    }
    __syncthreads();
    const int cb = wave * (16 * DLTN);
    for (int s = 0; s < nslab; ++s) {
        const int buf = s & 1;
        if (s + 1 < nslab) fetch((s + 1) * BK);
        if constexpr (P == 2) {
#pragma unroll
            for (int ks = 0; ks < BK / 32; ++ks) {
                h8x bf[DLTN];
#pragma unroll
                for (int j = 0; j < DLTN; ++j) bf[j] = *(const h8x*)&Bs[buf][cb + 16 * j + lr][32 * ks + 8 * lk];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const h8x af = *(const h8x*)&As[buf][16 * i + lr][32 * ks + 8 * lk];
#pragma unroll
                    for (int j = 0; j < DLTN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf[j], acc[i][j], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                T bf[DLTN];
#pragma unroll
                for (int j = 0; j < DLTN; ++j) bf[j] = Bs[buf][kk + lk][cb + 16 * j + lr];
#pragma unroll
                for (int i = 0; i < TM; ++i) {
                    const T af = As[buf][kk + lk][16 * i + lr];
#pragma unroll
                    for (int j = 0; j < DLTN; ++j) {
                        if constexpr (P == 0)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf[j], acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af, bf[j], acc[i][j], 0, 0, 0);
                    }
                }
            }
        }
        if (s + 1 < nslab) stash(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < DLTN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const long long row = m0 + 16 * i + (P == 0 ? lk + 4 * r : 4 * lk + r);
                const long long col = n0 + cb + 16 * j + lr;
                if (row < g.M && col < g.N) {
                    OT* c = C + row * g.ldc + col;
                    if constexpr (TO == 0) {
                        const double x = (double)acc[i][j][r];
                        *c = g.accumulate ? *c + x : x;
                    } else {
                        const float x = (float)acc[i][j][r];
                        *c = (OT)(g.accumulate ? (float)*c + x : x);
                    }
                }
            }
}

template <int P, int TO, int TM, bool BT>
void launch_tm(const DflArgs& a, int mtiles, int nbatch, hipStream_t s) {
    dim3 grid((unsigned)((a.N + DBN - 1) / DBN), (unsigned)mtiles, (unsigned)nbatch);
    if (a.vec) hipLaunchKernelGGL((dfl_kernel<P, TO, TM, BT, true>), grid, dim3(DNT), 0, s, a);
    else hipLaunchKernelGGL((dfl_kernel<P, TO, TM, BT, false>), grid, dim3(DNT), 0, s, a);
}

template <int P, int TO, bool BT = false>
void launch_p(const DflArgs& a, int tm, int mtiles, int nbatch, hipStream_t s) {
    switch (tm) {
        case 1: launch_tm<P, TO, 1, BT>(a, mtiles, nbatch, s); break;
        case 2: launch_tm<P, TO, 2, BT>(a, mtiles, nbatch, s); break;
        case 3: launch_tm<P, TO, 3, BT>(a, mtiles, nbatch, s); break;
        case 4: launch_tm<P, TO, 4, BT>(a, mtiles, nbatch, s); break;
        case 5: launch_tm<P, TO, 5, BT>(a, mtiles, nbatch, s); break;
        case 6: launch_tm<P, TO, 6, BT>(a, mtiles, nbatch, s); break;
        case 7: launch_tm<P, TO, 7, BT>(a, mtiles, nbatch, s); break;
        default: launch_tm<P, TO, 8, BT>(a, mtiles, nbatch, s); break;
    }
}

// ---------------------------------------------------------------------------
// BF16 operands, both k-contiguous:  C[m][n] (+)= sum_k A[m][k] Bt[n][k]  on v_mfma_f32_32x32x16_bf16.
// K is a list of nseg segments of seglen elements (segment g of row m at A + m lda + g segA, of row n
// at Bt + n ldb + g segB), so that step 2 reads B^Q rows straight from the factor, one segment per
// auxiliary function.  Workgroup tile (64 WM) x 128 from 4 waves in 2 x 2, each (32 WM) x 64 as WM x 2
// blocks of 32 x 32; slabs of 32 k.  Both tiles go from HBM into LDS by buffer loads (16 bytes a lane,
// no registers): one load fills 1 KB, 16 rows of 64 bytes, and lane i fetches the chunk (of 8 k) that
// belongs at LDS position (row i/4, slot i%4) under the swizzle slot = chunk ^ ((row / 4) % 4), which
// lets 16 lanes reading one chunk of 16 consecutive rows hit 16 different bank groups.  Every offset
// is per lane and relative to a per-workgroup descriptor that ends at the tile's last valid element:
// rows past M or N and chunks past a segment's end get an offset past the descriptor and read as zero,
// so partial slabs and tiles need no masking.  Chunks never straddle a segment (seglen % 8 == 0).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void* lds_ptr_t;
typedef float f16x __attribute__((ext_vector_type(16)));

struct DfbArgs {
    const __bf16* A; long long lda, bA0, bA1, segA;
    const __bf16* Bt; long long ldb, bB0, bB1, segB;
    void* C; long long ldc, bC0, bC1;
    long long m_off;
    int M, N, nseg, seglen, nb0;
    int accumulate;
};

constexpr unsigned DFB_OOR = 0xFFFFFFF0u;  // an offset past every descriptor of this kernel

// WM x WN blocks of 32 x 32 per wave; WAR waves along the rows and 4 / WAR along the columns; NST
// pipeline stages (slab t copied NST - 1 slabs ahead); OCC workgroups per CU for the register budget.
template <int WM, int WN, int WAR, int NST, int OCC, int TO>
__global__ __launch_bounds__(256, OCC) void dfb_kernel(DfbArgs g) {
    constexpr int WAC = 4 / WAR;
    constexpr int BM = 32 * WM * WAR, BN = 32 * WN * WAC;
    constexpr int LA = BM / 16, LB = BN / 16;  // 1 KB loads per slab and tile
    static_assert(WAR * WAC == 4 && LA % 4 == 0 && LB % 4 == 0, "every wave issues the same number of loads");
    static_assert(NST == 2 || NST == 3, "two or three stages");
    constexpr int SE = (BM + BN) * 32;  // one stage: the A tile, then the B tile
    // separate arrays per stage, so that the compiler tells the copies into one stage from the reads of
    // another and waits for the copies only where asked
    __shared__ __attribute__((aligned(16))) __bf16 S0[SE], S1[SE], S2[NST == 3 ? SE : 8];
    int tx, ty, tz;
    {  // XCD-contiguous ranges of the tile order (column tiles, then row tiles, then batches)
        const unsigned long long gx = gridDim.x, gy = gridDim.y;
        const unsigned long long total = gx * gy * gridDim.z;
        const unsigned long long H = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
        const unsigned long long per = total / 8, rem = total % 8, x = H % 8, j = H / 8;
        const unsigned long long L = x * per + (x < rem ? x : rem) + j;
        tx = (int)(L % gx);
        ty = (int)((L / gx) % gy);
        tz = (int)(L / (gx * gy));
    }
    const int b0 = tz % g.nb0, b1 = tz / g.nb0;
    const long long m0 = g.m_off + (long long)ty * BM, n0 = (long long)tx * BN;
    const int rows = (int)min((long long)BM, (long long)g.M - m0), cols = (int)min((long long)BN, (long long)g.N - n0);
    const long long kext = (long long)(g.nseg - 1);
    const __bf16* Ab = g.A + b0 * g.bA0 + b1 * g.bA1 + m0 * g.lda;
    const __bf16* Bb = g.Bt + b0 * g.bB0 + b1 * g.bB1 + n0 * g.ldb;
    const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Ab, (short)0, (int)(((rows - 1) * g.lda + kext * g.segA + g.seglen) * 2), 0x00020000);
    const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
        (void*)Bb, (short)0, (int)(((cols - 1) * g.ldb + kext * g.segB + g.seglen) * 2), 0x00020000);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // this lane's row and chunk in each of the wave's loads (fixed for the kernel)
    constexpr int NA = LA / 4, NB = LB / 4;
    unsigned rowa[NA], rowb[NB];
    int cha[NA], chb[NB];
#pragma unroll
    for (int t = 0; t < NA; ++t) {
        const int r = 16 * (wave + 4 * t) + (lane >> 2);
        rowa[t] = (unsigned)(r * g.lda * 2);
        cha[t] = (lane & 3) ^ ((r >> 2) & 3);
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const int r = 16 * (wave + 4 * t) + (lane >> 2);
        rowb[t] = (unsigned)(r * g.ldb * 2);
        chb[t] = (lane & 3) ^ ((r >> 2) & 3);
    }
    // a slab past the last one (seg == nseg) is copied as zeros: every offset past the descriptor
    auto issue = [&](__bf16(&St)[SE], int seg, int e0) {
        const unsigned sa = (unsigned)((seg * g.segA + e0) * 2), sb = (unsigned)((seg * g.segB + e0) * 2);
        const int lim = seg < g.nseg ? g.seglen : 0;  // chunks at or past lim read as zero
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            const int e = e0 + 8 * cha[t];
            const unsigned off = e < lim ? rowa[t] + sa + 16u * cha[t] : DFB_OOR;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr_t)&St[512 * (wave + 4 * t)], 16, off, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < NB; ++t) {
            const int e = e0 + 8 * chb[t];
            const unsigned off = e < lim ? rowb[t] + sb + 16u * chb[t] : DFB_OOR;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, (lds_ptr_t)&St[BM * 32 + 512 * (wave + 4 * t)], 16, off, 0, 0,
                                                     0);
        }
    };
    f16x acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int wr0 = (wave / WAC) * 32 * WM, wc0 = (wave % WAC) * 32 * WN;
    const int fr = lane & 31, fk = lane >> 5;
    // Rows of a fragment start at multiples of 32, so a row's swizzle is that of its lane (fr / 4 % 4).
    const int sw = (fr >> 2) & 3;
    // per 16-deep step: the fragments of WM row blocks and WN column blocks, then their WM WN products
    auto compute = [&](const __bf16(&St)[SE]) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int co = 8 * ((2 * ks + fk) ^ sw);
            h8x aq[WM], bq[WN];
#pragma unroll
            for (int j = 0; j < WN; ++j) bq[j] = *(const h8x*)&St[BM * 32 + 32 * (wc0 + 32 * j + fr) + co];
#pragma unroll
            for (int i = 0; i < WM; ++i) aq[i] = *(const h8x*)&St[32 * (wr0 + 32 * i + fr) + co];
#pragma unroll
            for (int i = 0; i < WM; ++i)
#pragma unroll
                for (int j = 0; j < WN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aq[i], bq[j], acc[i][j], 0, 0, 0);
        }
    };
    const int nsl = (g.seglen + 31) / 32, nslab = g.nseg * nsl;
    // slab t covers segment t / nsl, elements 32 (t % nsl) .. of it; advanced without a division
    int seg = 0, e0 = 0;
    auto next = [&] {
        e0 += 32;
        if (e0 >= g.seglen) { e0 = 0; ++seg; }
    };
    // Slab t lives in stage t % NST and is copied NST - 1 slabs ahead.  After slab t each wave waits until
    // only the copies of the slabs after t + 1 are outstanding (loads complete in issue order), then the
    // barrier makes slab t + 1 visible to all.  The last steps copy zero slabs into stages that are not
    // read again, so that every step has the same shape and the compiler's wait analysis sees no branch.
    constexpr int NL = NA + NB;
    static_assert((NST - 2) * NL < 16, "vmcnt immediate");
    // s_waitcnt immediates: vmcnt(n) with expcnt and lgkmcnt left at their maxima (no wait on them)
    constexpr int WAIT_STEP = (NST - 2) * NL | (0x7 << 4) | (0xF << 8), WAIT_0 = (0x7 << 4) | (0xF << 8);
    // the barrier alone: __syncthreads() would also wait for every copy in flight (its release fence
    // covers the copies into LDS).  The empty asm statements keep the compiler from moving LDS reads
    // across it.
    auto barrier = [] {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    auto step = [&](const __bf16(&Sc)[SE], __bf16(&Sn)[SE]) {
        issue(Sn, seg, e0);
        next();
        compute(Sc);
        __builtin_amdgcn_s_waitcnt(WAIT_STEP);
        barrier();
    };
    issue(S0, seg, e0);
    next();
    if constexpr (NST == 3) {
        issue(S1, seg, e0);
        next();
    }
    __builtin_amdgcn_s_waitcnt(WAIT_STEP);
    barrier();
    int t = 0;
    if constexpr (NST == 2) {
        for (; t + 2 <= nslab; t += 2) {
            step(S0, S1);
            step(S1, S0);
        }
        if (t < nslab) step(S0, S1);
    } else {
        for (; t + 3 <= nslab; t += 3) {
            step(S0, S2);
            step(S1, S0);
            step(S2, S1);
        }
        if (t < nslab) step(S0, S2);
        if (t + 1 < nslab) step(S1, S0);
    }
    __builtin_amdgcn_s_waitcnt(WAIT_0);
    // accumulator element r of lane l: row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
    typedef typename Out<TO>::T OT;
    OT* C = (OT*)g.C + b0 * g.bC0 + b1 * g.bC1;
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int lr = wr0 + 32 * i + 8 * (r >> 2) + 4 * fk + (r & 3);
                const int lc = wc0 + 32 * j + fr;
                if (lr < rows && lc < cols) {
                    OT* c = C + (m0 + lr) * g.ldc + n0 + lc;
                    if constexpr (TO == 0) {
                        const double x = (double)acc[i][j][r];
                        *c = g.accumulate ? *c + x : x;
                    } else {
                        *c = (OT)acc[i][j][r];
                    }
                }
            }
}

// can the k-contiguous BF16 kernel take this product?  (16-byte chunks that never straddle a segment,
// per-tile byte extents within the 32-bit descriptor range)
bool dfb_ok(const DfbArgs& a, int bm) {
    const auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    const long long ext = (long long)(a.nseg - 1);
    return a.seglen % 8 == 0 && a.lda % 8 == 0 && a.ldb % 8 == 0 && a.segA % 8 == 0 && a.segB % 8 == 0 &&
           a.bA0 % 8 == 0 && a.bA1 % 8 == 0 && a.bB0 % 8 == 0 && a.bB1 % 8 == 0 && al(a.A) && al(a.Bt) &&
           ((bm - 1) * a.lda + ext * a.segA + a.seglen) * 2 < (1LL << 31) &&
           (127 * a.ldb + ext * a.segB + a.seglen) * 2 < (1LL << 31);
}

template <int WM, int WN, int WAR, int NST, int OCC, int TO>
void dfb_launch(const DfbArgs& a, int nbatch, hipStream_t s) {
    constexpr int BM = 32 * WM * WAR, BN = 32 * WN * (4 / WAR);
    const long long rows_per_launch = 65535LL * BM;
    for (long long r0 = 0; r0 < a.M; r0 += rows_per_launch) {
        DfbArgs b = a;
        b.m_off = r0;
        b.M = (int)std::min<long long>(a.M, r0 + rows_per_launch);
        const long long rows = b.M - r0;
        dim3 grid((unsigned)((a.N + BN - 1) / BN), (unsigned)((rows + BM - 1) / BM), (unsigned)nbatch);
        hipLaunchKernelGGL((dfb_kernel<WM, WN, WAR, NST, OCC, TO>), grid, dim3(256), 0, s, b);
        LAUNCHCHK();
    }
}

// 256 x 128 workgroup tiles (4 x 2 blocks per wave), or 128 x 128 (2 x 2) where 256-row tiles would pad M
// more; two stages, two workgroups per CU.  Measured against the alternatives at v = 600, X = 1800, 200
// rows: three stages, and 512 x 128 tiles with 4 x 4 blocks per wave at one workgroup per CU, were within
// -2% .. +16% of this choice.
template <int TO>
void dfb_gemm(DfbArgs a, int nb1, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0) return;
    const int nbatch = a.nb0 * nb1;
    if (nbatch <= 0 || nbatch > 65535) fail(-1, "dfladder: batch count out of range");
    if (((a.M + 255) / 256) * 256 <= ((a.M + 127) / 128) * 128) dfb_launch<4, 2, 2, 2, 2, TO>(a, nbatch, s);
    else dfb_launch<2, 2, 2, 2, 2, TO>(a, nbatch, s);
}

// dst[m][j][i] = src[m][i][j], m < nb, n x n blocks of BF16
__global__ void transpose_bf16_kernel(unsigned short* dst, const unsigned short* src, int n, int nb) {
    __shared__ unsigned short t[32][33];
    const long long m = blockIdx.z;
    const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
    const unsigned short* S = src + m * (long long)n * n;
    unsigned short* D = dst + m * (long long)n * n;
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int i = i0 + r, j = j0 + threadIdx.x;
        if (i < n && j < n) t[r][threadIdx.x] = S[(long long)i * n + j];
    }
    __syncthreads();
    for (int r = threadIdx.y; r < 32; r += 8) {
        const int j = j0 + r, i = i0 + threadIdx.x;
        if (i < n && j < n) D[(long long)j * n + i] = t[threadIdx.x][r];
    }
}

int elem_bytes(int p) { return p == 0 ? 8 : p == 1 ? 4 : 2; }

// C = A B (or C += A B) over nbatch = nb0 * nb1 batches; out_prec selects C's type
// (0 FP64, 1 FP32, 2 BF16; for P = 0 only 0).  Rows are cut into launches of at most
// 65535 row tiles.
void dfl_gemm(int P, int out_prec, DflArgs a, int nb1, hipStream_t s, bool bt = false) {
    if (a.M <= 0 || a.N <= 0) return;
    const int nbatch = a.nb0 * nb1;
    if (nbatch <= 0 || nbatch > 65535) fail(-1, "dfladder: batch count out of range");
    if (bt && (P != 2 || a.kin <= 0)) fail(-1, "dfladder: transposed B operand is BF16 only");
    const int W = 16 / elem_bytes(P);
    const auto al = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    a.vec = (a.K % W == 0 && (bt ? (a.kin % W == 0 && a.ldbq % W == 0) : a.N % W == 0) && a.lda % W == 0 &&
             a.ldb % W == 0 && a.bA0 % W == 0 && a.bA1 % W == 0 && a.bB0 % W == 0 && a.bB1 % W == 0 && al(a.A) &&
             al(a.B)) ? 1 : 0;
    // rows: as few tiles as possible, each as short as M allows (<= 128 rows)
    int mt = (int)std::min<long long>(((long long)a.M + 127) / 128, 65535);
    const long long rows_per_launch = (long long)mt * 128;
    for (long long r0 = 0; r0 < a.M; r0 += rows_per_launch) {
        DflArgs b = a;
        b.m_off = r0;
        const long long rows = std::min<long long>(a.M - r0, rows_per_launch);
        const int mtiles = (int)((rows + 127) / 128);
        const int tm = (int)((rows + 16LL * mtiles - 1) / (16LL * mtiles));
        b.M = (int)std::min<long long>(a.M, r0 + rows);  // rows below M handled by this launch
        if (P == 0) launch_p<0, 0>(b, tm, mtiles, nbatch, s);
        else if (P == 1 && out_prec == 0) launch_p<1, 0>(b, tm, mtiles, nbatch, s);
        else if (P == 1) launch_p<1, 1>(b, tm, mtiles, nbatch, s);
        else if (out_prec == 0) launch_p<2, 0, true>(b, tm, mtiles, nbatch, s);
        else launch_p<2, 2, true>(b, tm, mtiles, nbatch, s);
        LAUNCHCHK();
    }
}
}  // namespace

namespace {
// upper-triangle pair index of (i, j), i <= j < o
__device__ inline long long pair_index(int i, int j, int o) { return (long long)i * o - (long long)i * (i - 1) / 2 + (j - i); }

// Tp[p(i,j)] = T[i][j] for i <= j   (blocks of vv)
__global__ void pairs_gather_kernel(double* Tp, const double* T, int o, long long vv) {
    const int i = blockIdx.y / o, j = blockIdx.y % o;
    if (j < i) return;
    const double* src = T + ((long long)i * o + j) * vv;
    double* dst = Tp + pair_index(i, j, o) * vv;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < vv; t += (long long)gridDim.x * blockDim.x)
        dst[t] = src[t];
}

// L[i][j] = Lp[p(i,j)], L[j][i] = Lp[p(i,j)]^T for i <= j   (v x v blocks)
__global__ void pairs_scatter_kernel(double* L, const double* Lp, int o, int v) {
    const int i = blockIdx.y / o, j = blockIdx.y % o;
    if (j < i) return;
    const long long vv = (long long)v * v;
    const double* src = Lp + pair_index(i, j, o) * vv;
    double* dij = L + ((long long)i * o + j) * vv;
    double* dji = L + ((long long)j * o + i) * vv;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < vv; t += (long long)gridDim.x * blockDim.x) {
        const long long a = t / v, b = t % v;
        dij[t] = src[t];
        if (i != j) dji[b * v + a] = src[t];
    }
}
}  // namespace

long long df_ladder_chunk(int M, int v, int X, long long v_elems) {
    const long long per = (long long)M * v * v;
    long long q = std::max<long long>(1, v_elems / std::max<long long>(per, 1));
    q = std::min<long long>(q, X);
    q = std::min<long long>(q, std::max(1, 65535 / std::max(M, 1)));
    return std::max<long long>(q, 1);
}

void df_ladder(int prec, int M, int v, int X, const void* Bvv, const void* Z, double* C, bool accumulate, void* V,
               long long v_elems, hipStream_t s) {
    if (g_dry) return;
    if (M <= 0 || v <= 0) return;
    if (M > 65535) fail(-1, "dfladder: too many rows");
    const long long vv = (long long)v * v;
    if (X <= 0) {
        if (!accumulate) k_fill(C, (long long)M * vv, 0.0, s);
        return;
    }
    // BF16 reads both B operands as [n][k] (16-byte LDS stores): step 1 from Z transposed per row
    // (kept at the end of the buffer), step 2 from B^Q itself, which is symmetric
    const bool bt = prec == 2;
    const long long zt_elems = bt ? (long long)M * vv + 8 : 0;
    const long long avail = v_elems - zt_elems;
    // BF16 on the k-contiguous kernel: the intermediate's segments start every vp elements, vp = v rounded
    // up to 64 (128 bytes) when the buffer allows, so that the row pieces one workgroup of step 1 writes
    // never share a cache line with another's
    const long long vround = (v + 63) / 64 * 64;
    const long long vp = (bt && v % 8 == 0 && avail >= (long long)M * v * vround) ? vround : v;
    const long long q = vp == v ? df_ladder_chunk(M, v, X, avail)
                                : std::max<long long>(1, std::min<long long>(std::min<long long>(X, avail / ((long long)M * v * vp)),
                                                                             std::max(1, 65535 / std::max(M, 1))));
    if (q * M * v * vp > avail) fail(-1, "dfladder: intermediate buffer too small");
    const int eb = elem_bytes(prec);
    const void* Zb = Z;
    if (bt) {
        unsigned short* Zt = (unsigned short*)V + ((v_elems - (long long)M * vv) & ~7LL);
        dim3 grid((unsigned)((v + 31) / 32), (unsigned)((v + 31) / 32), (unsigned)M);
        hipLaunchKernelGGL(transpose_bf16_kernel, grid, dim3(32, 8), 0, s, Zt, (const unsigned short*)Z, v, M);
        LAUNCHCHK();
        Zb = Zt;
    }
    for (long long Q0 = 0; Q0 < X; Q0 += q) {
        const int qn = (int)std::min<long long>(q, X - Q0);
        const char* Bq = (const char*)Bvv + Q0 * vv * eb;
        if (bt) {
            // both steps on the k-contiguous kernel when the shape allows
            DfbArgs s1{};
            s1.A = (const __bf16*)Bq; s1.lda = v; s1.bA0 = vv; s1.bA1 = 0; s1.segA = 0;
            s1.Bt = (const __bf16*)Zb; s1.ldb = v; s1.bB0 = 0; s1.bB1 = vv; s1.segB = 0;
            s1.C = V; s1.ldc = (long long)qn * vp; s1.bC0 = vp; s1.bC1 = (long long)qn * v * vp;
            s1.M = v; s1.N = v; s1.nseg = 1; s1.seglen = v; s1.nb0 = qn; s1.accumulate = 0;
            DfbArgs s2{};
            s2.A = (const __bf16*)V; s2.lda = (long long)qn * vp; s2.segA = vp;
            s2.Bt = (const __bf16*)Bq; s2.ldb = v; s2.segB = vv;
            s2.C = C; s2.ldc = v;
            s2.M = (int)((long long)M * v); s2.N = v; s2.nseg = qn; s2.seglen = v; s2.nb0 = 1;
            s2.accumulate = (accumulate || Q0 > 0) ? 1 : 0;
            if (dfb_ok(s1, 256) && dfb_ok(s2, 256)) {
                dfb_gemm<2>(s1, M, s);
                dfb_gemm<0>(s2, 1, s);
                continue;
            }
        }
        // step 1: V[m][a][Qi][e] = sum_c B^Q[a][c] Z_m[c][e]  (batch b0 = Qi, b1 = m)
        DflArgs a1{};
        a1.A = Bq; a1.lda = v; a1.bA0 = vv; a1.bA1 = 0;
        a1.B = Zb; a1.ldb = v; a1.bB0 = 0; a1.bB1 = vv; a1.ldbq = 0; a1.kin = v;
        a1.C = V; a1.ldc = (long long)qn * v; a1.bC0 = v; a1.bC1 = (long long)qn * vv;
        a1.M = v; a1.N = v; a1.K = v; a1.nb0 = qn;
        a1.accumulate = 0;
        dfl_gemm(prec, prec, a1, M, s, bt);
        // step 2: C[(m,a)][b] (+)= sum_(Qi,e) V[(m,a)][(Qi,e)] B^Q[e][b]
        DflArgs a2{};
        a2.A = V; a2.lda = (long long)qn * v;
        a2.B = Bq; a2.ldb = v; a2.ldbq = vv; a2.kin = v;
        a2.C = C; a2.ldc = v;
        a2.M = (int)((long long)M * v); a2.N = v; a2.K = qn * v; a2.nb0 = 1;
        a2.accumulate = (accumulate || Q0 > 0) ? 1 : 0;
        dfl_gemm(prec, 0, a2, 1, s, bt);
    }
}

}  // namespace adc3

namespace adc3 {
void k_pairs_gather(double* Tp, const double* T, int o, int v, hipStream_t s) {
    if (g_dry || o <= 0 || v <= 0) return;
    const long long vv = (long long)v * v;
    const unsigned gx = (unsigned)std::min<long long>((vv + 255) / 256, 1024);
    hipLaunchKernelGGL(pairs_gather_kernel, dim3(gx, (unsigned)(o * o)), dim3(256), 0, s, Tp, T, o, vv);
    LAUNCHCHK();
}

void k_pairs_scatter(double* L, const double* Lp, int o, int v, hipStream_t s) {
    if (g_dry || o <= 0 || v <= 0) return;
    const long long vv = (long long)v * v;
    const unsigned gx = (unsigned)std::min<long long>((vv + 255) / 256, 1024);
    hipLaunchKernelGGL(pairs_scatter_kernel, dim3(gx, (unsigned)(o * o)), dim3(256), 0, s, L, Lp, o, v);
    LAUNCHCHK();
}

void df_ladder_pairs(int o, int v, int X, const double* Bvv, const double* T, double* L, double* scratch, void* V,
                     long long v_elems, hipStream_t s) {
    if (g_dry) return;
    const long long vv = (long long)v * v, np = (long long)o * (o + 1) / 2;
    double* Tp = scratch;
    double* Lp = scratch + np * vv;
    const unsigned gx = (unsigned)std::min<long long>((vv + 255) / 256, 1024);
    hipLaunchKernelGGL(pairs_gather_kernel, dim3(gx, (unsigned)(o * o)), dim3(256), 0, s, Tp, T, o, vv);
    LAUNCHCHK();
    df_ladder(0, (int)np, v, X, Bvv, Tp, Lp, false, V, v_elems, s);
    hipLaunchKernelGGL(pairs_scatter_kernel, dim3(gx, (unsigned)(o * o)), dim3(256), 0, s, L, Lp, o, v);
    LAUNCHCHK();
}
}  // namespace adc3
