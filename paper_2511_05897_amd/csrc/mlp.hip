// Learned Davidson preconditioner: per-element MLP 6 -> 256 -> 256 -> 1 (GELU).
//
// The preconditioned step for root theta is t_e = a0_e (1 + u_e), a0_e = r_e/(D_e - theta)
// the Jacobi step and u = MLP(features).  Features of element e:
//   (D_e - theta)/(|theta|+1), r_e/rms(r), [e is 1p], e_a, e_b (0 for 1p), e_i (0 for 1p).
// Training minimises, per group of sampled elements of one residual vector, the
// scale-free 1 - cos^2(a, d) with a = a0 (1 + u) and d the ideal correction
// (converged vector minus current Ritz vector), averaged over the groups of a batch.
//
// Precision: training forward and the activation back-propagation run on FP32 matrix
// cores (FP32 master weights, FP32 accumulation); the weight-gradient reductions over
// samples run on FP64 matrix cores; Adam keeps FP64 moments.  Inference is one fused
// kernel per residual vector: FP32 first layer, BF16 matrix-core second layer with FP32
// accumulation, FP32 head, nothing but the step written back to HBM.
#include "internal.h"
#include <algorithm>
#include <cmath>
#include <vector>

namespace adc3 {

namespace {
constexpr int NF = 6, HD = 256;
constexpr int OFF_W1 = 0, OFF_B1 = NF * HD, OFF_W2 = OFF_B1 + HD, OFF_B2 = OFF_W2 + HD * HD, OFF_W3 = OFF_B2 + HD,
              OFF_B3 = OFF_W3 + HD, NPARAM = OFF_B3 + 1;
constexpr double C0 = 0.79788456080286535588;  // sqrt(2/pi)

__device__ inline double gelu(double z) { return 0.5 * z * (1.0 + tanh(C0 * (z + 0.044715 * z * z * z))); }
__device__ inline double gelu_d(double z) {
    double t = tanh(C0 * (z + 0.044715 * z * z * z));
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C0 * (1.0 + 3.0 * 0.044715 * z * z);
}
#define GS(i, n) for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)
inline unsigned nb(long long n) { long long b = (n + 255) / 256; return (unsigned)std::max<long long>(1, std::min<long long>(b, 8192)); }

// Z <- Z + b (pre-activation kept), H = GELU(Z)
__global__ void bias_gelu_kernel(double* Z, double* Hout, const float* b, long long n) {
    GS(t, n * HD) {
        double z = Z[t] + (double)b[t % HD];
        Z[t] = z;
        Hout[t] = gelu(z);
    }
}
// u_e = b3 + sum_j H[e][j] W3[j]
__global__ void head_kernel(const double* H, const float* w3, const float* b3, double* u, long long n) {
    GS(e, n) {
        double acc = (double)b3[0];
        const double* h = H + e * HD;
        for (int j = 0; j < HD; ++j) acc += h[j] * (double)w3[j];
        u[e] = acc;
    }
}
// per group: a = a0 (1+u); L_g = 1 - (a.d)^2/((a.a)(d.d)); du_e = dL/da_e * a0_e / G
__global__ void group_loss_kernel(const double* a0, const double* d, const double* u, int S, double invG,
                                  double* du, double* Lg) {
    const int g = blockIdx.x;
    const double* A0 = a0 + (long long)g * S;
    const double* Dd = d + (long long)g * S;
    const double* U = u + (long long)g * S;
    double p = 0, q = 0, nn = 0;
    for (int e = threadIdx.x; e < S; e += blockDim.x) {
        double a = A0[e] * (1.0 + U[e]);
        p += a * Dd[e];
        q += a * a;
        nn += Dd[e] * Dd[e];
    }
    __shared__ double sp[256], sq[256], sn[256];
    sp[threadIdx.x] = p; sq[threadIdx.x] = q; sn[threadIdx.x] = nn;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sp[threadIdx.x] += sp[threadIdx.x + o];
            sq[threadIdx.x] += sq[threadIdx.x + o];
            sn[threadIdx.x] += sn[threadIdx.x + o];
        }
        __syncthreads();
    }
    p = sp[0]; q = sq[0]; nn = sn[0];
    const bool ok = q > 0 && nn > 0;
    if (threadIdx.x == 0) Lg[g] = ok ? 1.0 - p * p / (q * nn) : 0.0;
    if (du) {
        const double c = ok ? -2.0 * p / (q * nn) * invG : 0.0, r = ok ? p / q : 0.0;
        for (int e = threadIdx.x; e < S; e += blockDim.x) {
            double a = A0[e] * (1.0 + U[e]);
            du[(long long)g * S + e] = c * (Dd[e] - r * a) * A0[e];
        }
    }
}
// dZ2[e][j] = du_e W3[j] gelu'(Z2[e][j])
__global__ void head_back_kernel(const double* du, const float* w3, const double* Z2, double* dZ2, long long n) {
    GS(t, n * HD) dZ2[t] = du[t / HD] * (double)w3[t % HD] * gelu_d(Z2[t]);
}
// dZ <- dZ * gelu'(Z)
__global__ void gelu_back_kernel(double* dZ, const double* Z, long long n) { GS(t, n * HD) dZ[t] *= gelu_d(Z[t]); }

__global__ void adam_kernel(float* w, const double* g, double* m, double* v, int n, double lr, double b1, double b2,
                            double eps, double c1, double c2) {
    GS(i, n) {
        double gi = g[i];
        double mi = b1 * m[i] + (1.0 - b1) * gi;
        double vi = b2 * v[i] + (1.0 - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] = (float)((double)w[i] - lr * (mi / c1) / (sqrt(vi / c2) + eps));
    }
}
__global__ void ones_kernel(double* x, long long n) { GS(i, n) x[i] = 1.0; }

// W2 as BF16, transposed to [out n][in k] so one lane's 8 consecutive k are 16 bytes
__global__ void w2t_bf16_kernel(const float* w, __bf16* wt) {
    GS(t, (long long)(HD * HD)) {
        const int n = (int)(t / HD), k = (int)(t % HD);
        wt[t] = (__bf16)w[OFF_W2 + k * HD + n];
    }
}

__device__ inline float gelu_fast(float z) {
    // z * sigmoid(2y), y = sqrt(2/pi)(z + 0.044715 z^3): the tanh form written with one exponential
    const float y2 = 2.0f * (float)C0 * (z + 0.044715f * z * z * z);
    return __fdividef(z, 1.0f + __expf(-y2));
}

// Fused learned preconditioner on one residual vector: per tile of 64 elements,
//   features -> layer 1 (FP32 FMA, 6 -> 256, GELU) -> BF16 tile in LDS
//   -> layer 2 on BF16 matrix cores (256 -> 256, FP32 accumulation) -> GELU -> head (FP32)
//   -> t_e = a0_e (1 + u_e);  a non-finite t_e falls back to a0_e and raises flag.
// Wave w owns output columns [64w, 64w+64) of layer 2 and keeps their W2 fragments
// (8 k-steps x 4 column tiles of 8 BF16) in registers for all tiles it visits.
constexpr int PT = 64;          // elements per tile
constexpr int H1LD = HD + 8;    // LDS row stride (BF16) of the layer-1 tile
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void precond_fused_kernel(const double* __restrict__ r, const double* __restrict__ D,
                                                            double theta, double rms, const double* __restrict__ eo,
                                                            const double* __restrict__ ev, int o, int v, long long N,
                                                            const float* __restrict__ w, const __bf16* __restrict__ w2t,
                                                            double* __restrict__ T, unsigned int* flag) {
    __shared__ __attribute__((aligned(16))) __bf16 h1s[PT][H1LD];
    __shared__ float Fs[PT][8];
    __shared__ double a0s[PT];
    __shared__ float us[4][PT];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const long long vv = (long long)v * v;
    // layer-1 column tid: weights and bias
    float w1c[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) w1c[f] = w[OFF_W1 + f * HD + tid];
    const float b1c = w[OFF_B1 + tid];
    // layer-2 fragments, bias and head weights of this wave's columns
    bf8v bw[4][HD / 32];
    float b2c[4], w3c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = 64 * wave + 16 * j + lr;
        b2c[j] = w[OFF_B2 + col];
        w3c[j] = w[OFF_W3 + col];
#pragma unroll
        for (int ks = 0; ks < HD / 32; ++ks) bw[j][ks] = *(const bf8v*)(w2t + (long long)col * HD + 32 * ks + 8 * lk);
    }
    const float b3 = w[OFF_B3];
    const float inv_rms = (float)(1.0 / rms), inv_th = (float)(1.0 / (fabs(theta) + 1.0));
    const long long ntiles = (N + PT - 1) / PT;
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long long e0 = tile * PT;
        if (tid < PT) {
            const long long e = e0 + tid;
            float f[NF] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            double a0 = 0.0;
            if (e < N) {
                const double re = r[e], de = D[e];
                double den = de - theta;
                if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
                a0 = re / den;
                f[0] = (float)(de - theta) * inv_th;
                f[1] = (float)re * inv_rms;
                if (e < v) {
                    f[2] = 1.f; f[3] = (float)ev[e];
                } else {
                    const long long q = e - v;
                    f[3] = (float)ev[(q / v) % v];
                    f[4] = (float)ev[q % v];
                    f[5] = (float)eo[q / vv];
                }
            }
#pragma unroll
            for (int c = 0; c < NF; ++c) Fs[tid][c] = f[c];
            a0s[tid] = a0;
        }
        __syncthreads();
        // layer 1: thread tid computes column tid of all 64 rows
        for (int row = 0; row < PT; ++row) {
            float z = b1c;
#pragma unroll
            for (int f = 0; f < NF; ++f) z += Fs[row][f] * w1c[f];
            h1s[row][tid] = (__bf16)gelu_fast(z);
        }
        __syncthreads();
        // layer 2: rows 16i + (4 lk + q), columns 64 wave + 16 j + lr
        f4v acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < HD / 32; ++ks) {
            bf8v af[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) af[i] = *(const bf8v*)&h1s[16 * i + lr][32 * ks + 8 * lk];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bw[j][ks], acc[i][j], 0, 0, 0);
        }
        // GELU, head partial sums over this lane's 4 columns, then over the 16 lanes of a row group
        float part[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float sacc = 0.f;
#pragma unroll
                for (int j = 0; j < 4; ++j) sacc += gelu_fast(acc[i][j][q] + b2c[j]) * w3c[j];
                part[i][q] = sacc;
            }
#pragma unroll
        for (int off = 1; off < 16; off <<= 1)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) part[i][q] += __shfl_xor(part[i][q], off, 64);
        if (lr == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) us[wave][16 * i + 4 * lk + q] = part[i][q];
        __syncthreads();
        if (tid < PT) {
            const long long e = e0 + tid;
            if (e < N) {
                const float u = b3 + us[0][tid] + us[1][tid] + us[2][tid] + us[3][tid];
                const double a0 = a0s[tid];
                double t = a0 * (1.0 + (double)u);
                if (!isfinite(t)) { atomicOr(flag, 1u); t = a0; }
                T[e] = t;
            }
        }
        __syncthreads();
    }
}

// sample index t of group g: splitmix64(seed + (g*S + t) * golden) mod N
__device__ inline long long sample_index(unsigned long long seed, int g, int S, int t, long long N) {
    unsigned long long z = seed + ((unsigned long long)g * S + t + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (long long)(z % (unsigned long long)N);
}
// features at the sampled elements of group g (same definitions as features_kernel); also the target there
__global__ void features_idx_kernel(const double* r, const double* D, double theta, double rms, const double* eo,
                                    const double* ev, int o, int v, unsigned long long seed, int g, int S, long long N,
                                    const double* xk, double* F, double* a0, double* xs) {
    const long long vv = (long long)v * v;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S) return;
    long long e = sample_index(seed, g, S, t, N);
    xs[t] = xk[e];
    double den = D[e] - theta;
    if (fabs(den) < 1e-8) den = den < 0 ? -1e-8 : 1e-8;
    a0[t] = r[e] / den;
    double* f = F + (long long)t * NF;
    f[0] = (D[e] - theta) / (fabs(theta) + 1.0);
    f[1] = r[e] / rms;
    if (e < v) {
        f[2] = 1.0; f[3] = ev[e]; f[4] = 0.0; f[5] = 0.0;
    } else {
        long long q = e - v;
        int i = (int)(q / vv), a = (int)((q / v) % v), b = (int)(q % v);
        f[2] = 0.0; f[3] = ev[a]; f[4] = ev[b]; f[5] = eo[i];
    }
}
}  // namespace

int mlp_nparam() { return NPARAM; }

// Scratch for forward/backward on n samples.
size_t mlp_scratch_elems(long long n) { return (size_t)(4 * n * HD + 4 * n + 2 * NPARAM + HD * 2 + 64); }

// u[n] = MLP(X[n][6]) on FP32 matrix cores (FP32 accumulation).
// Z1, H1, Z2, H2 are scratch [n][256] each (kept for the backward pass).
void mlp_forward(const float* w, const double* X, long long n, double* u, double* Z1, double* H1, double* Z2,
                 double* H2, hipStream_t s) {
    if (g_dry || n <= 0) return;
    const void* W1 = w + OFF_W1;
    const void* W2 = w + OFF_W2;
    GemmLP g1;
    g1.M = (int)n; g1.N = HD; g1.K = NF;
    g1.A = X; g1.sAm = NF; g1.sAk = 1;
    g1.B = W1; g1.sBk = HD; g1.sBn = 1;
    g1.C = Z1; g1.sCm = HD; g1.sCn = 1;
    gemm_lp(g1, 1, s);
    hipLaunchKernelGGL(bias_gelu_kernel, dim3(nb(n * HD)), dim3(256), 0, s, Z1, H1, w + OFF_B1, n);
    GemmLP g2;
    g2.M = (int)n; g2.N = HD; g2.K = HD;
    g2.A = H1; g2.sAm = HD; g2.sAk = 1;
    g2.B = W2; g2.sBk = HD; g2.sBn = 1;
    g2.C = Z2; g2.sCm = HD; g2.sCn = 1;
    gemm_lp(g2, 1, s);
    hipLaunchKernelGGL(bias_gelu_kernel, dim3(nb(n * HD)), dim3(256), 0, s, Z2, H2, w + OFF_B2, n);
    hipLaunchKernelGGL(head_kernel, dim3(nb(n)), dim3(256), 0, s, H2, w + OFF_W3, w + OFF_B3, u, n);
    LAUNCHCHK();
}

// Loss (and, if grad != null, the gradient [NPARAM] in FP64) of a batch of G groups of S samples.
// X [G*S][6], a0 [G*S], d [G*S].  scratch from mlp_scratch_elems(G*S).
double mlp_loss_grad(const float* w, const double* X, const double* a0, const double* d, int G, int S, double* grad,
                     double* scratch, double* Lg_host, hipStream_t s) {
    if (g_dry) return 0.0;
    const long long n = (long long)G * S;
    double* Z1 = scratch;
    double* H1 = Z1 + n * HD;
    double* Z2 = H1 + n * HD;
    double* H2 = Z2 + n * HD;
    double* u = H2 + n * HD;
    double* du = u + n;
    double* ones = du + n;
    double* Lg = ones + n;
    mlp_forward(w, X, n, u, Z1, H1, Z2, H2, s);
    hipLaunchKernelGGL(group_loss_kernel, dim3(G), dim3(256), 0, s, a0, d, u, S, 1.0 / G, grad ? du : nullptr, Lg);
    LAUNCHCHK();
    if (grad) {
        hipLaunchKernelGGL(ones_kernel, dim3(nb(n)), dim3(256), 0, s, ones, n);
        // head: dW3 = H2^T du, db3 = sum du
        gemm_rm(1, HD, (int)n, 1.0, du, 1, true, H2, HD, false, 0.0, grad + OFF_W3, HD, s);
        gemm_rm(1, 1, (int)n, 1.0, du, 1, true, ones, 1, false, 0.0, grad + OFF_B3, 1, s);
        // dZ2 (reuses H2's storage after dW3 is formed: keep order on the stream)
        double* dZ2 = H2;
        hipLaunchKernelGGL(head_back_kernel, dim3(nb(n * HD)), dim3(256), 0, s, du, w + OFF_W3, Z2, dZ2, n);
        LAUNCHCHK();
        gemm_rm(HD, HD, (int)n, 1.0, H1, HD, true, dZ2, HD, false, 0.0, grad + OFF_W2, HD, s);
        gemm_rm(1, HD, (int)n, 1.0, ones, 1, true, dZ2, HD, false, 0.0, grad + OFF_B2, HD, s);
        // dH1 = dZ2 W2^T on FP32 matrix cores, then dZ1 = dH1 * gelu'(Z1)
        double* dZ1 = H1;  // H1 no longer needed after dW2
        GemmLP gb;
        gb.M = (int)n; gb.N = HD; gb.K = HD;
        gb.A = dZ2; gb.sAm = HD; gb.sAk = 1;
        gb.B = w + OFF_W2; gb.sBk = 1; gb.sBn = HD;  // B(k,n) = W2[n][k]
        gb.C = dZ1; gb.sCm = HD; gb.sCn = 1;
        gemm_lp(gb, 1, s);
        hipLaunchKernelGGL(gelu_back_kernel, dim3(nb(n * HD)), dim3(256), 0, s, dZ1, Z1, n);
        LAUNCHCHK();
        gemm_rm(NF, HD, (int)n, 1.0, X, NF, true, dZ1, HD, false, 0.0, grad + OFF_W1, HD, s);
        gemm_rm(1, HD, (int)n, 1.0, ones, 1, true, dZ1, HD, false, 0.0, grad + OFF_B1, HD, s);
    }
    std::vector<double> h(G);
    HIPCHK(hipMemcpyAsync(h.data(), Lg, G * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double L = 0;
    for (int g = 0; g < G; ++g) L += h[g];
    if (Lg_host) for (int g = 0; g < G; ++g) Lg_host[g] = h[g];
    return L / G;
}

void mlp_adam(float* w, const double* grad, double* m, double* v, double lr, int step, hipStream_t s) {
    if (g_dry) return;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
    hipLaunchKernelGGL(adam_kernel, dim3(nb(NPARAM)), dim3(256), 0, s, w, grad, m, v, NPARAM, lr, b1, b2, eps, c1, c2);
    LAUNCHCHK();
}

// W2 in the BF16 transposed layout of the fused preconditioner (wt: HD*HD BF16)
void mlp_weights_bf16(const float* w, unsigned short* wt, hipStream_t s) {
    if (g_dry) return;
    hipLaunchKernelGGL(w2t_bf16_kernel, dim3(nb(HD * HD)), dim3(256), 0, s, w, (__bf16*)wt);
    LAUNCHCHK();
}

// t = learned preconditioner applied to residual r of root theta (fused kernel); flag set on fallback
void mlp_precondition(const double* r, const double* D, double theta, double rms, const double* eo, const double* ev,
                      int o, int v, long long N, const float* w, const unsigned short* wt, double* T,
                      unsigned int* flag, hipStream_t s) {
    if (g_dry || N <= 0) return;
    const long long ntiles = (N + PT - 1) / PT;
    const unsigned grid = (unsigned)std::min<long long>(ntiles, 1024);
    hipLaunchKernelGGL(precond_fused_kernel, dim3(grid), dim3(256), 0, s, r, D, theta, rms, eo, ev, o, v, N, w,
                       (const __bf16*)wt, T, flag);
    LAUNCHCHK();
}

void mlp_features_idx(const double* r, const double* D, double theta, double rms, const double* eo, const double* ev,
                      int o, int v, unsigned long long seed, int g, int S, long long N, const double* xk, double* F,
                      double* a0, double* xs, hipStream_t s) {
    if (g_dry || S <= 0) return;
    hipLaunchKernelGGL(features_idx_kernel, dim3((S + 255) / 256), dim3(256), 0, s, r, D, theta, rms, eo, ev, o, v,
                       seed, g, S, N, xk, F, a0, xs);
    LAUNCHCHK();
}


}  // namespace adc3
