// Elementwise and data-movement kernels (HBM-bound; grid-stride, coalesced writes).
#include "internal.h"

namespace adc3 {

namespace {
constexpr int NT = 256;
inline unsigned nblocks(long long n) {
    long long b = (n + NT - 1) / NT;
    if (b > 8192) b = 8192;
    return (unsigned)(b < 1 ? 1 : b);
}
#define GRID_STRIDE(i, n) for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)
// Kernels over nblk blocks of v*v elements: blocks along y (grid-stride beyond 65535), the v*v elements of
// a block along x, so that the per-element index arithmetic is 32-bit.
#define BLOCK_ROWS(blk, nblk) for (long long blk = blockIdx.y; blk < (nblk); blk += gridDim.y)
#define BLOCK_COLS(r, vv) for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < (vv); r += gridDim.x * blockDim.x)
inline dim3 block_grid(long long nblk, long long vv) {
    long long gx = (vv + NT - 1) / NT;
    if (gx > 1024) gx = 1024;
    long long gy = nblk < 1 ? 1 : nblk;
    if (gy > 65535) gy = 65535;
    return dim3((unsigned)(gx < 1 ? 1 : gx), (unsigned)gy);
}

__global__ void fill_kernel(double* x, long long n, double v) { GRID_STRIDE(i, n) x[i] = v; }
__global__ void copy_kernel(double* d, const double* s, long long n) { GRID_STRIDE(i, n) d[i] = s[i]; }
__global__ void axpby_kernel(double* y, const double* x, long long n, double a, double b) {
    GRID_STRIDE(i, n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

struct P4 { int d[4]; int perm[4]; };

// Permutes for the two cases of the innermost axes (input axis 3 and the input axis that becomes the
// output's axis 3):
//   * the same axis: element per thread, 32-bit index arithmetic (both sides contiguous);
//   * different axes X, Y: 32 x 32 tiles of (X, Y) transposed through LDS so that reads run along X and
//     writes along Y; the other two axes P, Q come from the grid.
struct P4T {
    int d[4];
    long long st[4], os[4];  // input strides, output strides, both indexed by input axis
    int X, Y, P, Q;
    unsigned q0, q1;  // same-innermost case: output strides of the first two output axes / d[3]
};

__global__ void permute4_same_kernel(double* out, const double* in, P4T p, unsigned n, double alpha, double beta) {
    // output order of the input axes: o0 o1 o2 then axis 3
    const unsigned d3 = (unsigned)p.d[3];
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const unsigned i3 = t % d3, r = t / d3;
        // r enumerates the other three axes in output order (p.X, p.Y, p.P: decreasing output stride)
        const unsigned a0 = r / p.q0, r1 = r - a0 * p.q0;
        const unsigned a1 = r1 / p.q1, a2 = r1 - a1 * p.q1;
        long long off = i3;
        off += (long long)a0 * p.st[p.X] + (long long)a1 * p.st[p.Y] + (long long)a2 * p.st[p.P];
        const double v = alpha * in[off];
        out[t] = (beta == 0.0) ? v : v + beta * out[t];
    }
}

__global__ __launch_bounds__(256) void permute4_tile_kernel(double* out, const double* in, P4T p, int nty,
                                                            double alpha, double beta) {
    __shared__ double tile[32][33];
    const int tx = blockIdx.x / nty, ty = blockIdx.x % nty;
    const long long bin = (long long)blockIdx.y * p.st[p.P] + (long long)blockIdx.z * p.st[p.Q];
    const long long bout = (long long)blockIdx.y * p.os[p.P] + (long long)blockIdx.z * p.os[p.Q];
    const int x0 = tx * 32, y0 = ty * 32;
    const int dx = p.d[p.X], dy = p.d[p.Y];
    {
        const int x = x0 + threadIdx.x;
        for (int j = threadIdx.y; j < 32; j += 8) {
            const int y = y0 + j;
            if (x < dx && y < dy) tile[j][threadIdx.x] = in[bin + (long long)y * p.st[p.Y] + x];
        }
    }
    __syncthreads();
    {
        const int y = y0 + threadIdx.x;
        for (int j = threadIdx.y; j < 32; j += 8) {
            const int x = x0 + j;
            if (x < dx && y < dy) {
                const long long o = bout + (long long)x * p.os[p.X] + y;
                const double v = alpha * tile[threadIdx.x][j];
                out[o] = (beta == 0.0) ? v : v + beta * out[o];
            }
        }
    }
}
__global__ void permute4_kernel(double* out, const double* in, P4 p, double alpha, double beta) {
    // output dims
    long long od[4], is[4];
    long long st[4];
    st[3] = 1; st[2] = p.d[3]; st[1] = (long long)p.d[3] * p.d[2]; st[0] = st[1] * p.d[1];
    for (int k = 0; k < 4; ++k) { od[k] = p.d[p.perm[k]]; is[k] = st[p.perm[k]]; }
    long long n = od[0] * od[1] * od[2] * od[3];
    GRID_STRIDE(t, n) {
        long long r = t;
        long long i3 = r % od[3]; r /= od[3];
        long long i2 = r % od[2]; r /= od[2];
        long long i1 = r % od[1]; r /= od[1];
        long long i0 = r;
        double v = alpha * in[i0 * is[0] + i1 * is[1] + i2 * is[2] + i3 * is[3]];
        out[t] = (beta == 0.0) ? v : v + beta * out[t];
    }
}

__global__ void split_B_kernel(const double* B, int X, int o, int v, double* Boo, double* Bov, double* Bvv) {
    const int n = o + v;
    long long tot = (long long)X * n * n;
    GRID_STRIDE(t, tot) {
        long long Q = t / ((long long)n * n);
        int r = (int)(t % ((long long)n * n));
        int p = r / n, q = r % n;
        double x = B[t];
        if (p < o && q < o) Boo[(Q * o + p) * o + q] = x;
        else if (p < o && q >= o) Bov[(Q * o + p) * v + (q - o)] = x;
        else if (p >= o && q >= o) Bvv[(Q * v + (p - o)) * v + (q - o)] = x;
    }
}

__global__ void amp_t_kernel(const double* ovov, const double* eo, const double* ev, int o, int v, double* T) {
    long long tot = (long long)o * o * v * v;
    GRID_STRIDE(t, tot) {
        int b = (int)(t % v); long long r = t / v;
        int a = (int)(r % v); r /= v;
        int j = (int)(r % o); int i = (int)(r / o);
        double g = ovov[(((long long)i * v + a) * o + j) * v + b];
        T[t] = g / (eo[i] + eo[j] - ev[a] - ev[b]);
    }
}

__global__ void div_d2_kernel(double* Y, const double* eo, const double* ev, int o, int v) {
    long long tot = (long long)o * o * v * v;
    GRID_STRIDE(t, tot) {
        int b = (int)(t % v); long long r = t / v;
        int a = (int)(r % v); r /= v;
        int j = (int)(r % o); int i = (int)(r / o);
        Y[t] /= (eo[i] + eo[j] - ev[a] - ev[b]);
    }
}

__global__ void div_d1_kernel(double* y, const double* eo, const double* ev, int o, int v) {
    long long tot = (long long)o * v;
    GRID_STRIDE(t, tot) {
        int a = (int)(t % v), i = (int)(t / v);
        y[t] /= (eo[i] - ev[a]);
    }
}

__global__ void comb_t_kernel(double* out, const double* T, long long nblk, int v, double ca, double cb) {
    long long vv = (long long)v * v, tot = nblk * vv;
    GRID_STRIDE(t, tot) {
        long long blk = t / vv;
        int r = (int)(t % vv), a = r / v, b = r % v;
        out[t] = ca * T[t] + cb * T[blk * vv + (long long)b * v + a];
    }
}

__global__ void copy2d_kernel(double* dst, long long ldd, const double* src, long long lds, long long rows,
                              long long cols, double a, double b) {
    long long tot = rows * cols;
    GRID_STRIDE(t, tot) {
        long long r = t / cols, c = t % cols;
        double v = a * src[r * lds + c];
        dst[r * ldd + c] = (b == 0.0) ? v : v + b * dst[r * ldd + c];
    }
}

__global__ void scale_rows_kernel(double* out, const double* in, const double* d, long long rows, long long cols) {
    long long tot = rows * cols;
    GRID_STRIDE(t, tot) out[t] = in[t] * d[t / cols];
}

__global__ void colsign_kernel(double* A, long long lda, int rows, int cols) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    double best = -1.0, sg = 1.0;
    for (int r = 0; r < rows; ++r) {
        double x = A[r * lda + c];
        if (fabs(x) > best) { best = fabs(x); sg = x < 0 ? -1.0 : 1.0; }
    }
    if (sg < 0)
        for (int r = 0; r < rows; ++r) A[r * lda + c] = -A[r * lda + c];
}

__global__ void residual_kernel(double* R, const double* AX, const double* X, const double* th, int nk, long long n) {
    long long tot = (long long)nk * n;
    GRID_STRIDE(t, tot) R[t] = AX[t] - th[t / n] * X[t];
}

__global__ void precond_kernel(double* T, const double* R, const double* D, const double* th, int nk, long long n) {
    long long tot = (long long)nk * n;
    GRID_STRIDE(t, tot) {
        double den = D[t % n] - th[t / n];
        if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
        T[t] = R[t] / den;
    }
}

__global__ void rscale_rows_kernel(double* T, int nn, long long n, const double* G, int ldg) {
    long long tot = (long long)nn * n;
    GRID_STRIDE(t, tot) {
        int j = (int)(t / n);
        double g = G[(long long)j * ldg + j];
        T[t] = (g > 0.0) ? T[t] / sqrt(g) : 0.0;
    }
}

__global__ void lowdin_coef_kernel(double* coef, const double* U, const double* w, int acc, int keep) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= acc * keep) return;
    int j = t / keep, q = t % keep;
    coef[t] = U[j * acc + q] / sqrt(w[q]);
}

__global__ void scale_vec_kernel(double* x, long long n, const double* f) {
    double a = f[0];
    GRID_STRIDE(t, n) x[t] *= a;
}

__global__ void check_B_kernel(const double* B, int X, int n, unsigned long long* out) {
    // out[0]: nonfinite flag, out[1]: max asym bits, out[2]: max |B| bits (non-negative doubles order as ints)
    long long tot = (long long)X * n * n;
    double masym = 0.0, mabs = 0.0;
    unsigned long long bad = 0;
    GRID_STRIDE(t, tot) {
        long long Q = t / ((long long)n * n);
        int r = (int)(t % ((long long)n * n)), p = r / n, q = r % n;
        double x = B[t];
        if (!isfinite(x)) bad = 1;
        mabs = fmax(mabs, fabs(x));
        if (p < q) masym = fmax(masym, fabs(x - B[Q * n * n + (long long)q * n + p]));
    }
    if (bad) atomicOr(&out[0], 1ull);
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(masym));
    atomicMax(&out[2], (unsigned long long)__double_as_longlong(mabs));
}

__global__ void z_to_x_kernel(const double* z, double* x, double* xt, long long nblk, int v) {
    const double is3 = 0.57735026918962576451;  // 1/sqrt(3)
    long long vv = (long long)v * v, tot = nblk * vv;
    GRID_STRIDE(t, tot) {
        long long blk = t / vv;
        int r = (int)(t % vv), a = r / v, b = r % v;
        double zab = z[t], zba = z[blk * vv + (long long)b * v + a];
        double s = 0.5 * (zab + zba), an = 0.5 * (zab - zba);
        double xab = s + an * is3, xba = s - an * is3;
        if (x) x[t] = xab;
        if (xt) xt[t] = 2.0 * xab - xba;
    }
}

__global__ void d_to_z_add_kernel(double* acc, const double* d, long long nblk, int v) {
    const double s3 = 1.73205080756887729353;
    const int vv = v * v;
    BLOCK_ROWS(blk, nblk) {
        const double* db = d + blk * vv;
        double* ab = acc + blk * vv;
        BLOCK_COLS(r, vv) {
            const int a = r / v, b = r - (r / v) * v;
            const double dab = db[r], dba = db[b * v + a];
            ab[r] += 0.5 * (dab + dba) + s3 * 0.5 * (dab - dba);
        }
    }
}

// Operands of the particle-hole terms, from z (blocks [n][j] of v x v, x = z_S + z_A/sqrt3 per block):
//   Y2[(n,a)][(j,d)] = x[n][j][a][d],  Y1 = 2 x[n][j][a][d] - x[n][j][d][a],  Y3[(n,a)][(j,d)] = x[n][j][d][a]
// rows (n,a) of length o*v, so that each term is one GEMM against a symmetric [(j,d)][(i,b)] matrix.
__global__ void ph_prep_kernel(const double* z, double* Y1, double* Y2, double* Y3, int nv, int o, int v) {
    const double is3 = 0.57735026918962576451;  // 1/sqrt(3)
    const int vv = v * v;
    const long long ov = (long long)o * v;
    BLOCK_ROWS(blk, (long long)nv * o) BLOCK_COLS(r, vv) {  // blk = n * o + j
        const int a = r / v, d = r - (r / v) * v;
        const int n = (int)(blk / o), j = (int)(blk % o);
        const double zad = z[blk * vv + r], zda = z[blk * vv + d * v + a];
        const double sy = 0.5 * (zad + zda), an = 0.5 * (zad - zda);
        const double xad = sy + an * is3, xda = sy - an * is3;
        const long long out = ((long long)n * v + a) * ov + (long long)j * v + d;
        Y1[out] = 2.0 * xad - xda;
        Y2[out] = xad;
        Y3[out] = xda;
    }
}

// acc[n][i][a][b] += S(d) + sqrt3 A(d) over (a,b), d[n][i][a][b] = C12[(n,a)][(i,b)] - C3[(n,b)][(i,a)]
__global__ void ph_fin_kernel(double* acc, const double* D, const double* E2, const double* E3, int nv, int o, int v) {
    const double s3 = 1.73205080756887729353;
    const int vv = v * v;
    const long long ov = (long long)o * v;
    BLOCK_ROWS(blk, (long long)nv * o) {  // blk = n * o + i
        const long long n = blk / o, i = blk % o;
        BLOCK_COLS(r, vv) {
            const int a = r / v, b = r - (r / v) * v;
            const long long ra = (n * v + a) * ov + i * v, rb = (n * v + b) * ov + i * v;
            const double dab = D[ra + b] - E2[ra + b] - E3[rb + a];
            const double dba = D[rb + a] - E2[rb + a] - E3[ra + b];
            acc[blk * vv + r] += 0.5 * (dab + dba) + s3 * 0.5 * (dab - dba);
        }
    }
}

__global__ void k0_add_kernel(double* s2, const double* z, const double* eo, const double* ev, int o, int v,
                              int nvec, long long ld) {
    const int vv = v * v;
    BLOCK_ROWS(blk, (long long)nvec * o) {  // blk = vec * o + i
        const long long vec = blk / o;
        const int i = (int)(blk % o);
        const long long base = vec * ld + (long long)i * vv;
        const double ei = eo[i];
        BLOCK_COLS(r, vv) {
            const int a = r / v, b = r - (r / v) * v;
            s2[base + r] += (ev[a] + ev[b] - ei) * z[base + r];
        }
    }
}

__global__ void symmetrize_kernel(double* A, int n) {
    long long tot = (long long)n * n;
    GRID_STRIDE(t, tot) {
        int i = (int)(t / n), j = (int)(t % n);
        if (i < j) {
            double m = 0.5 * (A[t] + A[(long long)j * n + i]);
            A[t] = m;
            A[(long long)j * n + i] = m;
        }
    }
}

__global__ void mirror_cols_kernel(double* G, int ld, int m0, int nc) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int rows = m0 + nc;
    if (t >= rows * nc) return;
    int i = t / nc, j = t % nc;
    if (i >= m0 && i - m0 >= j) return;  // new-new block: keep the upper copy, mirror below
    G[(long long)(m0 + j) * ld + i] = G[(long long)i * ld + m0 + j];
}

__global__ void add_diag_kernel(double* A, const double* d, int n) {
    GRID_STRIDE(i, n) A[(long long)i * n + i] += d[i];
}

// diag[0..v) = diag(M11); diag[v + (i*v + a)*v + b] = K0 + (level>=3) K1 diagonal in z coordinates
__global__ void diag_adc_kernel(double* diag, const double* M11, const double* eo, const double* ev,
                                const double* Bvv, const double* oovv, const double* ovov, int o, int v,
                                int X, int level, double x1) {
    const double s3 = 1.73205080756887729353;
    long long vv = (long long)v * v;
    GRID_STRIDE(t, vv) {
        int a = (int)(t / v), b = (int)(t % v);
        if (b == 0) diag[a] = M11[(long long)a * v + a];
        double aabb = 0.0, abab = 0.0;
        if (level >= 3) {
            for (int Q = 0; Q < X; ++Q) {
                const double* BQ = Bvv + (long long)Q * vv;
                aabb += BQ[(long long)a * v + a] * BQ[(long long)b * v + b];
                double x = BQ[(long long)a * v + b];
                abab += x * x;
            }
        }
        const double al = 0.5 + 0.5 * s3, be = 0.5 - 0.5 * s3;
        const double ga = 0.5 + 0.5 / s3, de = 0.5 - 0.5 / s3;
        for (int i = 0; i < o; ++i) {
            double d = ev[a] + ev[b] - eo[i];
            if (level >= 3) {
                double aaii = oovv[(((long long)i * o + i) * v + a) * v + a];
                double bbii = oovv[(((long long)i * o + i) * v + b) * v + b];
                double aiia = ovov[(((long long)i * v + a) * o + i) * v + a];
                double biib = ovov[(((long long)i * v + b) * o + i) * v + b];
                if (a == b) {
                    d += x1 * (aabb - 2.0 * aaii + aiia);
                } else {
                    double kabab = aabb - bbii - aaii + 2.0 * biib;
                    double kbaba = aabb - aaii - bbii + 2.0 * aiia;
                    double kabba = abab - biib;
                    double kbaab = abab - aiia;
                    d += x1 * (al * ga * kabab + al * de * kabba + be * ga * kbaab + be * de * kbaba);
                }
            }
            diag[v + ((long long)i * v + a) * v + b] = d;
        }
    }
}
// ---- fixed-shape block Davidson: convergence and masking decided on the device ----
// directions j < m with valid[j] == 0 are decoupled: their row and column of the Gram matrix are
// zeroed and their diagonal set above every eigenvalue of the valid block (its Gershgorin bound plus a
// margin), so their Ritz values sort after every real one without swamping the eigensolver's norms;
// cnt[0] = number of valid directions.  One workgroup.
__global__ void mask_gram_kernel(double* G, int m, const double* valid, double* cnt) {
    __shared__ double bnd[256];
    double b = -INFINITY;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        if (valid[i] == 0.0) continue;
        double r = G[(long long)i * m + i];
        for (int j = 0; j < m; ++j)
            if (j != i && valid[j] != 0.0) r += fabs(G[(long long)i * m + j]);
        b = fmax(b, r);
    }
    bnd[threadIdx.x] = b;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) bnd[threadIdx.x] = fmax(bnd[threadIdx.x], bnd[threadIdx.x + h]);
        __syncthreads();
    }
    const double top = bnd[0];
    const double shift = isfinite(top) ? top + 1.0 + fabs(top) : 1.0;
    __syncthreads();
    for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
        const int i = t / m, j = t % m;
        if (valid[i] == 0.0 || valid[j] == 0.0) G[t] = (i == j) ? shift : 0.0;
    }
    if (threadIdx.x == 0) {
        int n = 0;
        for (int i = 0; i < m; ++i) n += valid[i] != 0.0;
        cnt[0] = (double)n;
    }
}

// one workgroup: per root k, rn = sqrt(Gw[k][k]), converged when rn <= conv and |th - thold| <= conv;
// active[k] = !converged; thold = th; status = [all converged, all finite, rn[nroots], th[nroots],
// active[nroots]]
__global__ void dav_status_kernel(const double* Gw, int nroots, const double* th, double* thold, double conv,
                                  double* active, double* status) {
    __shared__ unsigned char okf[64], finf[64];
    for (int k = threadIdx.x; k < nroots; k += blockDim.x) {
        const double rn = sqrt(fmax(Gw[(long long)k * nroots + k], 0.0));
        const double w = th[k];
        const bool fin = isfinite(rn) && isfinite(w);
        const bool ok = fin && rn <= conv && fabs(w - thold[k]) <= conv;
        active[k] = ok ? 0.0 : 1.0;
        thold[k] = w;
        status[2 + k] = rn;
        status[2 + nroots + k] = w;
        status[2 + 2 * nroots + k] = ok ? 0.0 : 1.0;
        okf[k] = ok;
        finf[k] = fin;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nconv = 0, nfin = 0;
        for (int k = 0; k < nroots; ++k) { nconv += okf[k]; nfin += finf[k]; }
        status[0] = nconv == nroots ? 1.0 : 0.0;
        status[1] = nfin == nroots ? 1.0 : 0.0;
    }
}

// rows j of T[nn][n] with active[j] == 0 set to zero
__global__ void rows_mask_kernel(double* T, int nn, long long n, const double* active) {
    const long long tot = (long long)nn * n;
    GRID_STRIDE(t, tot) {
        if (active[t / n] == 0.0) T[t] = 0.0;
    }
}

// Loewdin coefficients over all nn directions: column q = U[:, q] / sqrt(w[q]) if w[q] > thr, else 0;
// valid[q] = (w[q] > thr)
__global__ void lowdin_masked_kernel(double* coef, const double* U, const double* w, int nn, double thr,
                                     double* valid) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * nn) return;
    const int q = t % nn;
    const bool keep = w[q] > thr && isfinite(w[q]);
    coef[t] = keep ? U[t] / sqrt(w[q]) : 0.0;
    if (t < nn) valid[t] = (w[t] > thr && isfinite(w[t])) ? 1.0 : 0.0;
}

__global__ void block_gather_kernel(double* thg, double* actg, double* rows, int ncol, const double* th,
                                    const double* active, const double* R, long long ldr, const double* idx, int nb) {
    const long long tot = (long long)nb * ncol;
    GRID_STRIDE(t, tot) {
        const int r = (int)(t / ncol);
        rows[t] = R[(long long)idx[r] * ldr + t % ncol];
    }
    if (blockIdx.x == 0)
        for (int r = threadIdx.x; r < nb; r += blockDim.x) {
            thg[r] = th[(int)idx[r]];
            actg[r] = active[(int)idx[r]];
        }
}

__global__ void precond_idx_kernel(double* T, const double* R, const double* D, const double* th, const double* idx,
                                   int nb, long long n) {
    const long long tot = (long long)nb * n;
    GRID_STRIDE(t, tot) {
        const int r = (int)(t / n);
        const long long e = t - (long long)r * n;
        const int k = (int)idx[r];
        double den = D[e] - th[k];
        if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
        T[t] = R[(long long)k * n + e] / den;
    }
}

// after a Rayleigh-Ritz sorted ascending, the first cnt[0] Ritz vectors are the valid ones
__global__ void valid_first_kernel(double* valid, int n, const double* cnt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) valid[t] = t < (int)cnt[0] ? 1.0 : 0.0;
}
}  // namespace

void k_mask_gram(double* G, int m, const double* valid, double* cnt, hipStream_t s) {
    if (g_dry || m <= 0) return;
    hipLaunchKernelGGL(mask_gram_kernel, dim3(1), dim3(256), 0, s, G, m, valid, cnt);
    LAUNCHCHK();
}
void k_dav_status(const double* Gw, int nroots, const double* th, double* thold, double conv, double* active,
                  double* status, hipStream_t s) {
    if (g_dry || nroots <= 0) return;
    if (nroots > 64) fail(-1, "dav_status: at most 64 roots");
    hipLaunchKernelGGL(dav_status_kernel, dim3(1), dim3(64), 0, s, Gw, nroots, th, thold, conv, active, status);
    LAUNCHCHK();
}
void k_rows_mask(double* T, int nn, long long n, const double* active, hipStream_t s) {
    if (g_dry) return;
    const long long t = (long long)nn * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(rows_mask_kernel, dim3(nblocks(t)), dim3(NT), 0, s, T, nn, n, active);
    LAUNCHCHK();
}
void k_lowdin_masked(double* coef, const double* U, const double* w, int nn, double thr, double* valid,
                     hipStream_t s) {
    if (g_dry || nn <= 0) return;
    hipLaunchKernelGGL(lowdin_masked_kernel, dim3((nn * nn + 255) / 256), dim3(256), 0, s, coef, U, w, nn, thr,
                       valid);
    LAUNCHCHK();
}
void k_block_gather(double* thg, double* actg, double* rows, int ncol, const double* th, const double* active,
                    const double* R, long long ldr, const double* idx, int nb, hipStream_t s) {
    if (g_dry || nb <= 0) return;
    const int nc = rows ? ncol : 0;
    const long long t = std::max<long long>((long long)nb * nc, 1);
    hipLaunchKernelGGL(block_gather_kernel, dim3(nblocks(t)), dim3(NT), 0, s, thg, actg, rows, nc, th, active, R, ldr,
                       idx, nb);
    LAUNCHCHK();
}
void k_precond_idx(double* T, const double* R, const double* D, const double* theta, const double* idx, int nb,
                   long long n, hipStream_t s) {
    if (g_dry) return;
    const long long t = (long long)nb * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(precond_idx_kernel, dim3(nblocks(t)), dim3(NT), 0, s, T, R, D, theta, idx, nb, n);
    LAUNCHCHK();
}
void k_valid_first(double* valid, int n, const double* cnt, hipStream_t s) {
    if (g_dry || n <= 0) return;
    hipLaunchKernelGGL(valid_first_kernel, dim3((n + 255) / 256), dim3(256), 0, s, valid, n, cnt);
    LAUNCHCHK();
}

void k_fill(double* x, long long n, double v, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_kernel, dim3(nblocks(n)), dim3(NT), 0, s, x, n, v);
    LAUNCHCHK();
}
void k_copy(double* d, const double* src, long long n, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    hipLaunchKernelGGL(copy_kernel, dim3(nblocks(n)), dim3(NT), 0, s, d, src, n);
    LAUNCHCHK();
}
void k_axpby(double* y, const double* x, long long n, double a, double b, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    hipLaunchKernelGGL(axpby_kernel, dim3(nblocks(n)), dim3(NT), 0, s, y, x, n, a, b);
    LAUNCHCHK();
}
void k_permute4(double* out, const double* in, const int din[4], const int perm[4], double alpha, double beta,
                hipStream_t s) {
    if (g_dry) return;
    P4 p;
    long long n = 1;
    for (int k = 0; k < 4; ++k) { p.d[k] = din[k]; p.perm[k] = perm[k]; n *= din[k]; }
    if (n <= 0) return;
    // strides of each input axis in the input and in the output
    P4T t;
    long long ost[4];
    ost[3] = 1;
    for (int k = 2; k >= 0; --k) ost[k] = ost[k + 1] * din[perm[k + 1]];
    t.st[3] = 1;
    for (int k = 2; k >= 0; --k) t.st[k] = t.st[k + 1] * din[k + 1];
    for (int k = 0; k < 4; ++k) { t.d[k] = din[k]; t.os[perm[k]] = ost[k]; }
    const int X = 3, Y = perm[3];
    if (X != Y) {
        int others[2], no = 0;
        for (int a = 0; a < 4; ++a)
            if (a != X && a != Y) others[no++] = a;
        t.X = X; t.Y = Y; t.P = others[0]; t.Q = others[1];
        const int ntx = (din[X] + 31) / 32, nty = (din[Y] + 31) / 32;
        if ((long long)ntx * nty <= 0x7fffffffLL && din[t.P] <= 65535 && din[t.Q] <= 65535) {
            hipLaunchKernelGGL(permute4_tile_kernel, dim3((unsigned)(ntx * nty), (unsigned)din[t.P], (unsigned)din[t.Q]),
                               dim3(32, 8), 0, s, out, in, t, nty, alpha, beta);
            LAUNCHCHK();
            return;
        }
    } else if (n < 0x7fffffffLL) {
        // the other three axes in output order (decreasing output stride)
        int ax[3], na = 0;
        for (int k = 0; k < 3; ++k) ax[na++] = perm[k];
        t.X = ax[0]; t.Y = ax[1]; t.P = ax[2]; t.Q = 3;
        t.q0 = (unsigned)(ost[0] / din[3]);
        t.q1 = (unsigned)(ost[1] / din[3]);
        hipLaunchKernelGGL(permute4_same_kernel, dim3(nblocks(n)), dim3(NT), 0, s, out, in, t, (unsigned)n, alpha, beta);
        LAUNCHCHK();
        return;
    }
    hipLaunchKernelGGL(permute4_kernel, dim3(nblocks(n)), dim3(NT), 0, s, out, in, p, alpha, beta);
    LAUNCHCHK();
}
void k_split_B(const double* B, int X, int o, int v, double* Boo, double* Bov, double* Bvv, hipStream_t s) {
    if (g_dry) return;
    long long n = (long long)X * (o + v) * (o + v);
    if (n <= 0) return;
    hipLaunchKernelGGL(split_B_kernel, dim3(nblocks(n)), dim3(NT), 0, s, B, X, o, v, Boo, Bov, Bvv);
    LAUNCHCHK();
}
void k_amp_t(const double* ovov, const double* eo, const double* ev, int o, int v, double* T, hipStream_t s) {
    if (g_dry) return;
    long long n = (long long)o * o * v * v;
    hipLaunchKernelGGL(amp_t_kernel, dim3(nblocks(n)), dim3(NT), 0, s, ovov, eo, ev, o, v, T);
    LAUNCHCHK();
}
void k_div_d2(double* Y, const double* eo, const double* ev, int o, int v, hipStream_t s) {
    if (g_dry) return;
    long long n = (long long)o * o * v * v;
    hipLaunchKernelGGL(div_d2_kernel, dim3(nblocks(n)), dim3(NT), 0, s, Y, eo, ev, o, v);
    LAUNCHCHK();
}
void k_div_d1(double* y, const double* eo, const double* ev, int o, int v, hipStream_t s) {
    if (g_dry) return;
    long long n = (long long)o * v;
    hipLaunchKernelGGL(div_d1_kernel, dim3(nblocks(n)), dim3(NT), 0, s, y, eo, ev, o, v);
    LAUNCHCHK();
}
void k_comb_t(double* out, const double* T, long long nblk, int v, double a, double b, hipStream_t s) {
    if (g_dry) return;
    long long n = nblk * v * v;
    if (n <= 0) return;
    hipLaunchKernelGGL(comb_t_kernel, dim3(nblocks(n)), dim3(NT), 0, s, out, T, nblk, v, a, b);
    LAUNCHCHK();
}
void k_copy2d(double* dst, long long ldd, const double* src, long long lds, long long rows, long long cols,
              double a, double b, hipStream_t s) {
    if (g_dry) return;
    long long n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL(copy2d_kernel, dim3(nblocks(n)), dim3(NT), 0, s, dst, ldd, src, lds, rows, cols, a, b);
    LAUNCHCHK();
}
void k_scale_rows(double* out, const double* in, const double* d, long long rows, long long cols, hipStream_t s) {
    if (g_dry) return;
    long long n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL(scale_rows_kernel, dim3(nblocks(n)), dim3(NT), 0, s, out, in, d, rows, cols);
    LAUNCHCHK();
}
void k_colsign(double* A, long long lda, int rows, int cols, hipStream_t s) {
    if (g_dry) return;
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(colsign_kernel, dim3((cols + 255) / 256), dim3(256), 0, s, A, lda, rows, cols);
    LAUNCHCHK();
}
void k_residual(double* R, const double* AX, const double* X, const double* th, int nk, long long n, hipStream_t s) {
    if (g_dry) return;
    long long t = (long long)nk * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(residual_kernel, dim3(nblocks(t)), dim3(NT), 0, s, R, AX, X, th, nk, n);
    LAUNCHCHK();
}
// y[a] /= (lam[a] - th[0])  (denominators clamped away from 0 as in the diagonal step)
__global__ void div_shift_kernel(double* y, const double* lam, const double* th, int n) {
    GRID_STRIDE(t, (long long)n) {
        double den = lam[t] - th[0];
        if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
        y[t] /= den;
    }
}

void k_div_shift(double* y, const double* lam, const double* th, int n, hipStream_t s) {
    if (g_dry || n <= 0) return;
    hipLaunchKernelGGL(div_shift_kernel, dim3(nblocks(n)), dim3(NT), 0, s, y, lam, th, n);
    LAUNCHCHK();
}

// The exact 1p-block step of up to 16 vectors in one launch, one workgroup per vector j:
//   t1 = Q (diag(w) - theta_k)^-1 Q^T r1,   r1 = R[k][0:v], t1 -> T[tidx[j]][0:v],   k = kidx[j],
// with M11 = Q diag(w) Q^T (Q[k][n]: component k of eigenvector n), the shift floored as div_shift_kernel
// floors it.  Both products read Q from global memory (L2-resident, 8 v^2 bytes) with r1 and the scaled
// coefficients in LDS; sums in a fixed order (deterministic).
__global__ __launch_bounds__(1024) void precond_1p_kernel(Precond1p a) {
    extern __shared__ double sh[];
    const int j = blockIdx.x, k = a.kidx[j], v = a.v, tid = threadIdx.x;
    const double* r = a.R + (long long)k * a.N;
    double* t = a.T + (long long)a.tidx[j] * a.N;
    double* rs = sh;          // r1, then the scaled coefficients
    double* part = sh + v;    // [4][v] partial sums of Q^T r1 over k quarters
    for (int i = tid; i < v; i += 1024) rs[i] = r[i];
    __syncthreads();
    const int g = tid >> 8, n0 = tid & 255;
    const int kq = (v + 3) / 4, klo = g * kq, khi = min(v, klo + kq);
    for (int n = n0; n < v; n += 256) {
        double acc = 0.0;
        for (int kk = klo; kk < khi; ++kk) acc += rs[kk] * a.Q[(long long)kk * v + n];
        part[g * v + n] = acc;
    }
    __syncthreads();
    const double th = a.th[k];
    for (int n = tid; n < v; n += 1024) {
        const double y = ((part[n] + part[v + n]) + part[2 * v + n]) + part[3 * v + n];
        double den = a.w[n] - th;
        if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
        rs[n] = y / den;
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    for (int m = wave; m < v; m += 16) {
        double acc = 0.0;
        for (int n = lane; n < v; n += 64) acc += a.Q[(long long)m * v + n] * rs[n];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) t[m] = acc;
    }
}

void k_precond_1p(const Precond1p& a, hipStream_t s) {
    if (g_dry || a.nrow <= 0 || a.v <= 0) return;
    if (a.nrow > 16) fail(-1, "precond_1p: more than 16 vectors in one launch");
    const size_t lds = (size_t)5 * a.v * sizeof(double);
    if (a.v > PRECOND_1P_VMAX) fail(-1, "precond_1p: nvir too large for the LDS");
    hipLaunchKernelGGL(precond_1p_kernel, dim3((unsigned)a.nrow), dim3(1024), lds, s, a);
    LAUNCHCHK();
}

// T -= (s[0]/s[1]) B  (s[1] == 0: T unchanged)
__global__ void olsen_kernel(double* T, const double* B, const double* sc, long long n) {
    const double d = sc[1];
    const double e = d != 0.0 ? sc[0] / d : 0.0;
    GRID_STRIDE(t, n) T[t] -= e * B[t];
}

void k_olsen(double* T, const double* B, const double* sc, long long n, hipStream_t s) {
    if (g_dry || n <= 0) return;
    hipLaunchKernelGGL(olsen_kernel, dim3(nblocks(n)), dim3(NT), 0, s, T, B, sc, n);
    LAUNCHCHK();
}

void k_precond(double* T, const double* R, const double* D, const double* th, int nk, long long n, hipStream_t s) {
    if (g_dry) return;
    long long t = (long long)nk * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(precond_kernel, dim3(nblocks(t)), dim3(NT), 0, s, T, R, D, th, nk, n);
    LAUNCHCHK();
}
void k_scale_vec(double* x, long long n, const double* f, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    hipLaunchKernelGGL(scale_vec_kernel, dim3(nblocks(n)), dim3(NT), 0, s, x, n, f);
    LAUNCHCHK();
}
void k_rscale_rows(double* T, int nn, long long n, const double* G, int ldg, hipStream_t s) {
    if (g_dry) return;
    long long t = (long long)nn * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(rscale_rows_kernel, dim3(nblocks(t)), dim3(NT), 0, s, T, nn, n, G, ldg);
    LAUNCHCHK();
}
void k_lowdin_coef(double* coef, const double* U, const double* w, int acc, int keep, hipStream_t s) {
    if (g_dry) return;
    if (acc <= 0 || keep <= 0) return;
    hipLaunchKernelGGL(lowdin_coef_kernel, dim3((acc * keep + 255) / 256), dim3(256), 0, s, coef, U, w, acc, keep);
    LAUNCHCHK();
}
void k_check_B(const double* B, int X, int n, double* flags, hipStream_t s) {
    if (g_dry) return;
    HIPCHK(hipMemsetAsync(flags, 0, 3 * sizeof(double), s));
    long long t = (long long)X * n * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(check_B_kernel, dim3(nblocks(t)), dim3(NT), 0, s, B, X, n, (unsigned long long*)flags);
    LAUNCHCHK();
}
void k_z_to_x(const double* z, double* x, double* xt, long long nblk, int v, hipStream_t s) {
    if (g_dry) return;
    long long n = nblk * v * v;
    if (n <= 0) return;
    hipLaunchKernelGGL(z_to_x_kernel, dim3(nblocks(n)), dim3(NT), 0, s, z, x, xt, nblk, v);
    LAUNCHCHK();
}
void k_ph_prep(const double* z, double* Y1, double* Y2, double* Y3, int nv, int o, int v, hipStream_t s) {
    if (g_dry) return;
    long long n = (long long)nv * o * v * v;
    if (n <= 0) return;
    hipLaunchKernelGGL(ph_prep_kernel, block_grid((long long)nv * o, (long long)v * v), dim3(NT), 0, s, z, Y1, Y2, Y3, nv,
                       o, v);
    LAUNCHCHK();
}
void k_ph_fin(double* acc, const double* D, const double* E2, const double* E3, int nv, int o, int v, hipStream_t s) {
    if (g_dry) return;
    long long n = (long long)nv * o * v * v;
    if (n <= 0) return;
    hipLaunchKernelGGL(ph_fin_kernel, block_grid((long long)nv * o, (long long)v * v), dim3(NT), 0, s, acc, D, E2, E3, nv,
                       o, v);
    LAUNCHCHK();
}
void k_d_to_z_add(double* acc, const double* d, long long nblk, int v, hipStream_t s) {
    if (g_dry) return;
    long long n = nblk * v * v;
    if (n <= 0) return;
    hipLaunchKernelGGL(d_to_z_add_kernel, block_grid(nblk, (long long)v * v), dim3(NT), 0, s, acc, d, nblk, v);
    LAUNCHCHK();
}
void k_k0_add(double* s2, const double* z, const double* eo, const double* ev, int o, int v, int nvec,
              long long ld, hipStream_t s) {
    if (g_dry) return;
    long long n = (long long)o * v * v * nvec;
    if (n <= 0) return;
    hipLaunchKernelGGL(k0_add_kernel, block_grid((long long)nvec * o, (long long)v * v), dim3(NT), 0, s, s2, z, eo, ev, o,
                       v, nvec, ld);
    LAUNCHCHK();
}
void k_symmetrize(double* A, int n, hipStream_t s) {
    if (g_dry) return;
    long long nn = (long long)n * n;
    if (nn <= 0) return;
    hipLaunchKernelGGL(symmetrize_kernel, dim3(nblocks(nn)), dim3(NT), 0, s, A, n);
    LAUNCHCHK();
}
void k_mirror_cols(double* G, int ld, int m0, int nc, hipStream_t s) {
    if (g_dry) return;
    int n = (m0 + nc) * nc;
    if (n <= 0) return;
    hipLaunchKernelGGL(mirror_cols_kernel, dim3((n + 255) / 256), dim3(256), 0, s, G, ld, m0, nc);
    LAUNCHCHK();
}
void k_add_diag(double* A, const double* d, int n, hipStream_t s) {
    if (g_dry) return;
    if (n <= 0) return;
    hipLaunchKernelGGL(add_diag_kernel, dim3(nblocks(n)), dim3(NT), 0, s, A, d, n);
    LAUNCHCHK();
}
void k_diag_adc(double* diag, const double* M11, const double* eo, const double* ev, const double* Bvv,
                const double* oovv, const double* ovov, int o, int v, int X, int level, hipStream_t s, double x1) {
    if (g_dry) return;
    long long n = (long long)v * v;
    if (n <= 0) return;
    hipLaunchKernelGGL(diag_adc_kernel, dim3(nblocks(n)), dim3(NT), 0, s, diag, M11, eo, ev, Bvv, oovv, ovov, o,
                       v, X, level, x1);
    LAUNCHCHK();
}

}  // namespace adc3
