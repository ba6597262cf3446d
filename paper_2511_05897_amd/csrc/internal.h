// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace adc3 {

// dry run: allocations are counted, no device work is issued (workspace planning)
extern thread_local bool g_dry;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error {
    int status;
    std::string msg;
};
void set_error(const std::string& msg);
[[noreturn]] void fail(int status, const std::string& msg);

#define HIPCHK(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            ::adc3::fail(-3, std::string(#call) + ": " + hipGetErrorString(e_));           \
    } while (0)

#define LAUNCHCHK() HIPCHK(hipGetLastError())

// ---------------------------------------------------------------------------
// bump allocator over the caller's workspace; base == nullptr only counts bytes (the pointers it
// then hands out lie in a fake, never dereferenced range, so that offsets applied to them by the
// counting dry runs stay defined)
// ---------------------------------------------------------------------------
constexpr uintptr_t ARENA_COUNT_BASE = uintptr_t(1) << 44;
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    size_t peak = 0;
    template <class T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        size_t bytes = count * sizeof(T);
        used = off + bytes;
        if (used > peak) peak = used;
        if (base == nullptr) return reinterpret_cast<T*>(ARENA_COUNT_BASE + off);
        if (used > cap) fail(-2, "workspace too small: need at least " + std::to_string(used) + " bytes");
        return reinterpret_cast<T*>(base + off);
    }
    size_t mark() const { return used; }
    void release(size_t m) { used = m; }
};

// ---------------------------------------------------------------------------
// GEMM:  C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n)
// A(m,k) = A[bA0*b0 + bA1*b1 + m*sAm + k*sAk], likewise B, C; batch index
// b = b0 + nb0*b1 over nbatch = nb0*nb1.
// ---------------------------------------------------------------------------
struct Gemm {
    int M = 0, N = 0, K = 0;
    const double* A = nullptr; long long sAm = 0, sAk = 0, bA0 = 0, bA1 = 0;
    const double* B = nullptr; long long sBk = 0, sBn = 0, bB0 = 0, bB1 = 0;
    double* C = nullptr; long long sCm = 0, sCn = 0, bC0 = 0, bC1 = 0;
    int nb0 = 1, nb1 = 1;
    double alpha = 1.0, beta = 0.0;
    int Klast = -1;  // if >= 0: K of the batches with b0 == nb0-1 (ragged last K chunk)
};
void gemm(const Gemm& g, hipStream_t s, int tag = 0);
// as gemm, but a single GEMM with few output tiles splits K from K >= 512 on (gemm: K >= 4096)
void gemm_split(const Gemm& g, hipStream_t s, int tag = 0);
// reduced-precision GEMM, FP32 accumulation, FP64 C (see gemm_lp.hip):
// A FP64 (converted on load), B in the reduced type (prec 1: float, 2: bf16)
struct GemmLP {
    int M = 0, N = 0, K = 0;
    const double* A = nullptr; long long sAm = 0, sAk = 0;
    const float* Af = nullptr;  // if set (prec 1 only): A read as FP32 instead of A
    const void* B = nullptr; long long sBk = 0, sBn = 0;
    double* C = nullptr; long long sCm = 0, sCn = 0;
    double alpha = 1.0, beta = 0.0;
    long long bA = 0, bB = 0, bC = 0;  // per-K-chunk offsets (blockIdx.z), in elements
    int Klast = -1;                    // K of the last chunk if >= 0
};
void splitk_reduce(const double* part, int nchunk, int M, int N, double alpha, double beta, double* C,
                   long long sCm, long long sCn, hipStream_t s);
// part[c][m][n] = sum over K chunk c of A[m][k] B[n][k] for M <= 16, N <= 256 rows contiguous along K (row
// strides lda, ldb); returns the chunk count (0: nothing launched, shape or partial buffer unsuitable)
// both U_z products of a sigma pass in one stream over U [v][K] (v <= 256, M <= 16, 16-byte aligned rows):
// part1[c][m][a] = chunk c's share of sum_k r2[m][k] U[a][k] (sum with splitk_reduce over the returned chunk
// count), out2[m][k] = sum_a r1[m][a] U[a][k]; returns 0 with nothing launched when the shape does not fit
long long couple_fused(int M, int v, long long K, const double* U, long long ldu, const double* r2, long long ld2,
                       const double* r1, long long ld1, double* out2, long long ldo, double* part1,
                       long long partial_elems, hipStream_t s);
// the same with U_z in FP32 (widened to FP64 on load; ldu a multiple of 4)
long long couple_fused32(int M, int v, long long K, const float* U, long long ldu, const double* r2, long long ld2,
                         const double* r1, long long ld1, double* out2, long long ldo, double* part1,
                         long long partial_elems, hipStream_t s);
long long abt_skinny_chunks(int M, int N, long long K, long long partial_elems);
long long abt_skinny(int M, int N, long long K, const double* A, long long lda, const double* B, long long ldb,
                     double* part, long long partial_elems, hipStream_t s);
// sigma ladder (dedicated FP64 kernel): C = alpha Z G + beta C, K split into nchunk chunks
// whose partial sums go to partial[nchunk][M][N] (nchunk 1: direct)
bool ladder_supported(int M, int N, int K, const double* Z, long long ldz, const double* G, long long ldg,
                      const double* C, long long ldc);
int ladder_chunk_len(int K, int nchunk);
void ladder_rows(int M, int& tm, int& mtiles);
void ladder_gemm(int M, int N, int K, double alpha, const double* Z, long long ldz, const double* G, long long ldg,
                 double beta, double* C, long long ldc, int nchunk, double* partial, long long partial_elems,
                 hipStream_t s, int tag = 0);  // tag: 0 sigma ladder, 1 tuner trial, 2 other GEMM
// the same product with Z k-major (Zt[k][m], ldz >= M): both tiles copied HBM -> LDS by buffer loads.
// Each chunk must stay below 2^31 bytes: nchunk is raised to ladder_t_min_chunks (0: shape not
// supported).  Returns false, with nothing launched, when those chunks do not fit the partial buffer.
int ladder_t_min_chunks(int K, long long ldz, long long ldg);
bool ladder_t_supported(int M, int N, int K, const double* Zt, long long ldz, const double* G, long long ldg);
bool ladder_gemm_t(int M, int N, int K, double alpha, const double* Zt, long long ldz, const double* G, long long ldg,
                   double beta, double* C, long long ldc, int nchunk, double* partial, long long partial_elems,
                   hipStream_t s, int tag = 0);  // tag: 0 sigma ladder, 1 tuner trial, 2 other GEMM
// FP32 operands (FP32 accumulation, FP64 partial sums / output), Z k-major, ldz and ldg multiples of 4
int ladder_t32_min_chunks(int K, long long ldz, long long ldg);
bool ladder_t32_supported(int M, int N, int K, const float* Zt, long long ldz, const float* G, long long ldg);
bool ladder_gemm_t32(int M, int N, int K, double alpha, const float* Zt, long long ldz, const float* G, long long ldg,
                     double beta, double* C, long long ldc, int nchunk, double* partial, long long partial_elems,
                     hipStream_t s, int tag = 0);
bool ladder_lp_supported(int prec, int M, int N, int K, const void* Z, long long ldz, const void* G, long long ldg,
                         const double* C, long long ldc);
void ladder_gemm_lp(int prec, int M, int N, int K, double alpha, const void* Z, long long ldz, const void* G,
                    long long ldg, double beta, double* C, long long ldc, int nchunk, double* partial,
                    long long partial_elems, hipStream_t s, bool trial = false);
// chunk count for a ladder shape (prec 0 FP64, 1 FP32, 2 BF16, 3 FP64 / 4 FP32 with Z k-major), measured on first use
int ladder_tuned_chunks(int prec, int M, int N, int K, const void* Z, long long ldz, const void* G, long long ldg,
                        double* C, long long ldc, double* partial, long long partial_elems, hipStream_t s);
// ladder from the DF factor (dfladder.hip): C[m] (+)= sum_Q B^Q Z[m] B^Q for m < M, with Bvv [X][v][v]
// and Z [M][v][v] in the operand precision prec (0 FP64, 1 FP32, 2 BF16), C FP64 [M][v][v]; V is an
// intermediate of v_elems elements of that precision holding q*M*v*v for the chunk size q (BF16: plus
// M*v*v + 8 for Z transposed)
long long df_ladder_chunk(int M, int v, int X, long long v_elems);
void df_ladder(int prec, int M, int v, int X, const void* Bvv, const void* Z, double* C, bool accumulate, void* V,
               long long v_elems, hipStream_t s);
// FP64 ladder of amplitudes with T[j][i] = T[i][j]^T (o x o blocks of v x v): L[i][j] = sum_Q B^Q T[i][j] B^Q is
// formed for i <= j only and L[j][i] = L[i][j]^T; scratch holds 2 * o(o+1)/2 * v*v doubles.
// k_pairs_gather: Tp[p(i,j)] = T[i][j] for i <= j (v x v blocks, pairs row-major over i <= j);
// k_pairs_scatter: L[i][j] = Lp[p(i,j)], L[j][i] = Lp[p(i,j)]^T.
void df_ladder_pairs(int o, int v, int X, const double* Bvv, const double* T, double* L, double* scratch, void* V,
                     long long v_elems, hipStream_t s);
void k_pairs_gather(double* Tp, const double* T, int o, int v, hipStream_t s);
void k_pairs_scatter(double* L, const double* Lp, int o, int v, hipStream_t s);
extern thread_local double* g_gemm_scratch;
extern thread_local long long g_gemm_scratch_n;
void gemm_lp(const GemmLP& g, int prec, hipStream_t s, int tag = 0);
void k_to_lowp(void* dst, const double* src, long long n, int prec, hipStream_t s);
// scratch for split-K GEMMs issued by this thread while the guard lives
struct GemmScratch {
    double* prev;
    long long prev_n;
    GemmScratch(Arena& ws, long long n);
    ~GemmScratch();
};
constexpr long long GEMM_SCRATCH = 4LL << 20;  // doubles
// row-major helpers: C[M,N] (ldc) = alpha*op(A)op(B) + beta*C
void gemm_rm(int M, int N, int K, double alpha, const double* A, long long lda, bool transA,
             const double* B, long long ldb, bool transB, double beta, double* C, long long ldc,
             hipStream_t s, int tag = 0);

// ---------------------------------------------------------------------------
// profiling: HIP events around selected launches, on the launching stream
// ---------------------------------------------------------------------------
enum ProfKernel { PROF_LADDER = 0, PROF_SIGMA = 1, PROF_SETUP = 2, PROF_DAVIDSON = 3, PROF_EIG = 4, PROF_LADDER_LP = 5, PROF_N = 6 };
struct ProfScope {
    int k;
    hipStream_t s;
    double flops, bytes, bound_ms;  // bound_ms: the launch's roofline time, max(flops/peak, bytes/bandwidth)
    void* ev0 = nullptr;
    ProfScope(int kernel, hipStream_t stream, double flops, double bytes, double bound_ms = 0.0);
    ~ProfScope();
};

// ---------------------------------------------------------------------------
// elementwise / data movement
// ---------------------------------------------------------------------------
void k_fill(double* x, long long n, double v, hipStream_t s);
void k_copy(double* dst, const double* src, long long n, hipStream_t s);
void k_axpby(double* y, const double* x, long long n, double a, double b, hipStream_t s);  // y = a*x + b*y
// out[d0][d1][d2][d3] with out index permutation: out[i0][i1][i2][i3] = alpha*in[...] + beta*out
// perm[k] = which input axis becomes output axis k; in dims din[4]
void k_permute4(double* out, const double* in, const int din[4], const int perm[4], double alpha,
                double beta, hipStream_t s);
void k_split_B(const double* B, int X, int o, int v, double* Boo, double* Bov, double* Bvv, hipStream_t s);
// T[i][j][a][b] = ovov[i][a][j][b] / (eo_i + eo_j - ev_a - ev_b)
void k_amp_t(const double* ovov, const double* eo, const double* ev, int o, int v, double* T, hipStream_t s);
// Y[i][j][a][b] /= (eo_i + eo_j - ev_a - ev_b)
void k_div_d2(double* Y, const double* eo, const double* ev, int o, int v, hipStream_t s);
void k_div_d1(double* y, const double* eo, const double* ev, int o, int v, hipStream_t s);
// out = a*T + b*T^(ab swapped), T[n][v][v] blocks
void k_comb_t(double* out, const double* T, long long nblk, int v, double a, double b, hipStream_t s);
// dst[r*ldd + c] = a*src[r*lds + c] + b*dst[r*ldd + c]
void k_copy2d(double* dst, long long ldd, const double* src, long long lds, long long rows, long long cols,
              double a, double b, hipStream_t s);
void k_scale_rows(double* out, const double* in, const double* d, long long rows, long long cols, hipStream_t s);
// make the largest-|.| entry of each column of A[rows][cols] (row stride lda) positive
void k_colsign(double* A, long long lda, int rows, int cols, hipStream_t s);
// R[k][i] = AX[k][i] - theta[k] X[k][i]
void k_residual(double* R, const double* AX, const double* X, const double* theta, int nk, long long n, hipStream_t s);
// T[k][i] = R[k][i] / (D[i] - theta[k]) with |D - theta| >= floor
void k_precond(double* T, const double* R, const double* D, const double* theta, int nk, long long n, hipStream_t s);
void k_olsen(double* T, const double* B, const double* sc, long long n, hipStream_t s);  // T -= (sc[0]/sc[1]) B
void k_div_shift(double* y, const double* lam, const double* th, int n, hipStream_t s);  // y /= lam - th[0]
// exact 1p-block preconditioner step of nrow <= 16 vectors:
//   T[tidx[j]][0:v] = Q (diag(w) - th[kidx[j]])^-1 Q^T R[kidx[j]][0:v]   (rows of length N)
// (shift floored at 1e-8 as k_div_shift); 5 v doubles of LDS, v <= PRECOND_1P_VMAX
struct Precond1p {
    const double* R = nullptr; double* T = nullptr; long long N = 0;
    const double* Q = nullptr; const double* w = nullptr; const double* th = nullptr;
    int v = 0, nrow = 0;
    int kidx[16] = {}, tidx[16] = {};
};
constexpr int PRECOND_1P_VMAX = 1638;
void k_precond_1p(const Precond1p& a, hipStream_t s);
void k_scale_vec(double* x, long long n, const double* factor_dev, hipStream_t s);   // x *= factor[0]
// row j of T[nn][n] *= 1/sqrt(G[j*ldg + j])  (rows with G <= 0 are zeroed)
void k_rscale_rows(double* T, int nn, long long n, const double* G, int ldg, hipStream_t s);
// coef[j*keep + q] = U[j*acc + q] / sqrt(w[q]),  j < acc, q < keep
void k_lowdin_coef(double* coef, const double* U, const double* w, int acc, int keep, hipStream_t s);
// fixed-shape block Davidson helpers (no host decisions):
// G[m][m]: rows/columns of directions with valid[j] == 0 zeroed, their diagonal set above the valid
// block's Gershgorin bound; cnt[0] = number of valid directions
void k_mask_gram(double* G, int m, const double* valid, double* cnt, hipStream_t s);
// per root: rn = sqrt(Gw[k][k]), converged = rn <= conv && |th - thold| <= conv; active = !converged;
// thold = th; status = [all converged, all finite, rn[nroots], th[nroots], active[nroots]]  (one workgroup)
void k_dav_status(const double* Gw, int nroots, const double* th, double* thold, double conv, double* active,
                  double* status, hipStream_t s);
void k_rows_mask(double* T, int nn, long long n, const double* active, hipStream_t s);  // zero inactive rows
// the block of the roots idx[0..nb): thg[r] = th[idx[r]], actg[r] = active[idx[r]]; with rows != nullptr also
// rows[r][0..ncol) = R[idx[r]][0..ncol) (R rows of length ldr)
void k_block_gather(double* thg, double* actg, double* rows, int ncol, const double* th, const double* active,
                    const double* R, long long ldr, const double* idx, int nb, hipStream_t s);
// T[r] = R[idx[r]] / (D - th[idx[r]]) elementwise (the Jacobi step of root idx[r]), r < nb
void k_precond_idx(double* T, const double* R, const double* D, const double* theta, const double* idx, int nb,
                   long long n, hipStream_t s);
// coef[j*nn + q] = U[j*nn + q] / sqrt(w[q]) for w[q] > thr, else 0; valid[q] = w[q] > thr
void k_lowdin_masked(double* coef, const double* U, const double* w, int nn, double thr, double* valid,
                     hipStream_t s);
void k_valid_first(double* valid, int n, const double* cnt, hipStream_t s);  // valid[t] = t < cnt[0]
// flags[0] = 1 if any non-finite; flags[1] = max |B_Qpq - B_Qqp|; flags[2] = max |B|
void k_check_B(const double* B, int X, int n, double* flags, hipStream_t s);
// z -> x = z_S + z_A/sqrt3 and xt = 2x - x^T  (blocks of v*v)
void k_z_to_x(const double* z, double* x, double* xt, long long nblk, int v, hipStream_t s);
// acc += S(d) + sqrt3*A(d)
void k_d_to_z_add(double* acc, const double* d, long long nblk, int v, hipStream_t s);
// particle-hole terms: operands from z ([nv][o] blocks of v x v) as rows (n,a) x cols (j,d):
// Stored ladder in pair-symmetric (a <= b) and pair-antisymmetric (a < b) blocks, each padded to a
// leading dimension that is a multiple of 8 (sa_lp(v), sa_lm(v); the padding is zero).
long long sa_lp(int v);
long long sa_lm(int v);
// w+[m][lp] = z[c][d] + z[d][c] (c < d), z[c][c];  w-[m][lm] = z[c][d] - z[d][c]  (z rows of v*v, stride ldz)
void k_sa_pack(const double* z, long long ldz, int M, int v, double* Ws, double* Wa, hipStream_t s);
// out[m][a][b] = C+[(ab)] + C-[(ab)] (a < b), C+[(ba)] - C-[(ba)] (a > b), C+[(aa)]  (row stride ldo)
void k_sa_unpack(const double* Cs, const double* Ca, int M, int v, double* out, long long ldo, hipStream_t s);
// dst[c][r] = src[r][c] for r < rows, c < cols (tiled through LDS)
void k_transpose(const double* src, long long lds, int rows, long long cols, double* dst, long long ldd, hipStream_t s);
// G+ / G- rows (a,b), a in [a0, a0+na), b >= a, from (ac|bd) = Gf[((a-a0) v + c) ldf + (b-a0) v + d]
void k_sa_form(const double* Gf, long long ldf, int a0, int na, int v, double* Gp, double* Gm, hipStream_t s);
// zero the padding rows of G+ and G-
void k_sa_zero_pad_rows(double* Gp, double* Gm, int v, hipStream_t s);
// Y2 = x[n][j][a][d], Y1 = 2x[n][j][a][d] - x[n][j][d][a], Y3 = x[n][j][d][a]
void k_ph_prep(const double* z, double* Y1, double* Y2, double* Y3, int nv, int o, int v, hipStream_t s);
// acc[n][i][a][b] += S(d) + sqrt3 A(d), d[n][i][a][b] = D[(n,a)][(i,b)] - E2[(n,a)][(i,b)] - E3[(n,b)][(i,a)]
void k_ph_fin(double* acc, const double* D, const double* E2, const double* E3, int nv, int o, int v, hipStream_t s);
// sigma2 += K0 * z, K0[i][a][b] = ev_a + ev_b - eo_i;  z/sigma2 with vector stride ld
void k_k0_add(double* s2, const double* z, const double* eo, const double* ev, int o, int v, int nvec,
              long long ld, hipStream_t s);
void k_symmetrize(double* A, int n, hipStream_t s);   // A = (A + A^T)/2
// G[(m0+j)*ld + i] = G[i*ld + m0 + j] for i < m0 + nc, j < nc  (new columns mirrored into rows)
void k_mirror_cols(double* G, int ld, int m0, int nc, hipStream_t s);
void k_add_diag(double* A, const double* d, int n, hipStream_t s);
// diagonal of M; x1 scales the first-order 2p1h terms (level 3; sm-ADC)
void k_diag_adc(double* diag, const double* M11, const double* eo, const double* ev, const double* Bvv,
                const double* oovv, const double* ovov, int o, int v, int X, int level, hipStream_t s,
                double x1 = 1.0);

// ---------------------------------------------------------------------------
// reductions (deterministic, FP64)
// ---------------------------------------------------------------------------
// G[p][q] = sum_i X[p*ldx + i] * Y[q*ldy + i], p < np, q < nq  (G row stride ldg)
void k_dots(const double* X, long long ldx, int np, const double* Y, long long ldy, int nq, long long n,
            double* G, int ldg, double* partial, hipStream_t s);
size_t dots_partial_elems(int np, int nq, long long n);
// Y[q][i] = beta*Y[q][i] + alpha * sum_p C[p*ldc + q] * X[p][i]    (linear combination of rows)
void k_lincomb(double* Y, long long ldy, int nq, const double* X, long long ldx, int np, const double* C,
               int ldc, long long n, double alpha, double beta, hipStream_t s);

// ---------------------------------------------------------------------------
// symmetric eigensolvers (Jacobi, FP64)
// ---------------------------------------------------------------------------
// A[n][n] (destroyed) -> w[n] ascending, V[n][n] columns eigenvectors (row-major V[i*n+k])
void eig_small(double* A, int n, double* w, double* V, hipStream_t s);   // n <= 96, one workgroup
void eig_large(double* A, int n, double* w, double* V, double* scratch, hipStream_t s);
size_t eig_large_scratch(int n);
// nb independent matrices of order n, contiguous A[nb][n][n] (destroyed), w[nb][n], V[nb][n][n] (unsorted, as
// eig_large): the launches of each round serve the whole batch, each matrix stopping at its own convergence
void eig_batched(double* A, int n, int nb, double* w, double* V, double* scratch, hipStream_t s);
size_t eig_batched_scratch(int n, int nb);
// reorder eigenpairs descending (desc=1) or ascending and fix signs (largest |.| positive)
void k_sort_eig(double* w, double* V, int n, int desc, double* wtmp, double* Vtmp, hipStream_t s);

// learned preconditioner (mlp.hip)
int mlp_nparam();
size_t mlp_scratch_elems(long long n);
void mlp_forward(const float* w, const double* X, long long n, double* u, double* Z1, double* H1, double* Z2,
                 double* H2, hipStream_t s);
double mlp_loss_grad(const float* w, const double* X, const double* a0, const double* d, int G, int S, double* grad,
                     double* scratch, double* Lg_host, hipStream_t s);
void mlp_adam(float* w, const double* grad, double* m, double* v, double lr, int step, hipStream_t s);
void mlp_weights_bf16(const float* w, unsigned short* wt, hipStream_t s);
void mlp_precondition(const double* r, const double* D, double theta, double rms, const double* eo, const double* ev,
                      int o, int v, long long N, const float* w, const unsigned short* wt, double* T,
                      unsigned int* flag, hipStream_t s);
void mlp_features_idx(const double* r, const double* D, double theta, double rms, const double* eo, const double* ev,
                      int o, int v, unsigned long long seed, int g, int S, long long N, const double* xk, double* F,
                      double* a0, double* xs, hipStream_t s);

}  // namespace adc3
