// Two-operand tensor contraction expressed as one GEMM on the matrix cores.
//
//   out[...] = alpha * sum_K A[...] B[...] + beta * out[...]
//
// Labels are single letters; an operand has at most 4 axes.  Labels shared by A
// and B and absent from the output are contracted (K); labels of A in the output
// form the GEMM rows (M), labels of B in the output the columns (N).  An operand
// whose axes are already ordered [M..,K..] / [K..,M..] (resp. [K..,N..] /
// [N..,K..]) is used in place through strides; otherwise it is permuted once into
// a workspace buffer.  The output is written through strides when its axes read
// [M..,N..] or [N..,M..], else through a permuted temporary.
#include "internal.h"
#include "tensor.h"
#include <algorithm>
#include <cstring>

namespace adc3 {

thread_local bool g_dry = false;

namespace {
struct Parsed {
    std::string a, b, o;
};
Parsed parse(const char* spec) {
    Parsed p;
    const char* comma = std::strchr(spec, ',');
    const char* arrow = std::strstr(spec, "->");
    if (!comma || !arrow) fail(-1, std::string("ein2: bad spec ") + spec);
    p.a.assign(spec, comma);
    p.b.assign(comma + 1, arrow);
    p.o.assign(arrow + 2);
    return p;
}
long long prod_dims(const std::string& labels, const std::string& from, const int* dims) {
    long long n = 1;
    for (char c : labels) n *= dims[from.find(c)];
    return n;
}
// permutation that reorders `from` into `to` (to[k] = from[perm[k]])
void perm_of(const std::string& from, const std::string& to, int* perm) {
    for (size_t k = 0; k < to.size(); ++k) perm[k] = (int)from.find(to[k]);
}
// pad to 4D with leading unit axes
void permute_any(double* out, const double* in, const std::string& from, const int* dims, const std::string& to,
                 double alpha, double beta, hipStream_t s) {
    int d4[4] = {1, 1, 1, 1}, p4[4] = {0, 1, 2, 3};
    int nd = (int)from.size();
    int off = 4 - nd;
    for (int k = 0; k < nd; ++k) d4[off + k] = dims[k];
    int perm[4];
    perm_of(from, to, perm);
    for (int k = 0; k < nd; ++k) p4[off + k] = off + perm[k];
    for (int k = 0; k < off; ++k) p4[k] = k;
    k_permute4(out, in, d4, p4, alpha, beta, s);
}
}  // namespace

void ein2(Arena& ws, const char* spec, double alpha, const double* A, const int* adims, const double* B,
          const int* bdims, double beta, double* C, hipStream_t s) {
    Parsed p = parse(spec);
    std::string Ml, Nl, Kl;
    for (char c : p.o) {
        bool ina = p.a.find(c) != std::string::npos, inb = p.b.find(c) != std::string::npos;
        if (ina && inb) fail(-1, std::string("ein2: batch label unsupported in ") + spec);
        if (ina) Ml += c;
        else if (inb) Nl += c;
        else fail(-1, std::string("ein2: output label not in inputs: ") + spec);
    }
    for (char c : p.a)
        if (p.b.find(c) != std::string::npos && p.o.find(c) == std::string::npos) Kl += c;
    for (char c : p.b)
        if (p.o.find(c) == std::string::npos && p.a.find(c) == std::string::npos)
            fail(-1, std::string("ein2: dangling label in ") + spec);
    for (char c : p.a)
        if (p.o.find(c) == std::string::npos && p.b.find(c) == std::string::npos)
            fail(-1, std::string("ein2: dangling label in ") + spec);
    // output dims
    int odims[4];
    for (size_t k = 0; k < p.o.size(); ++k) {
        char c = p.o[k];
        size_t ia = p.a.find(c);
        odims[k] = (ia != std::string::npos) ? adims[ia] : bdims[p.b.find(c)];
    }
    const long long M = prod_dims(Ml, p.a, adims), N = prod_dims(Nl, p.b, bdims), K = prod_dims(Kl, p.a, adims);
    size_t mark = ws.mark();
    Gemm g;
    g.M = (int)M; g.N = (int)N; g.K = (int)K;
    g.alpha = alpha;
    if (M > 2147483647LL || N > 2147483647LL || K > 2147483647LL) fail(-1, "ein2: dimension too large");
    // A large contraction gets row-major B and output and a contiguous A (a permute of each is cheap
    // next to the GEMM), so that it runs on the ladder tiles: A k-major ([K..,M..], both tiles copied
    // straight into LDS; K in consecutive ranges when one launch's 32-bit offsets cannot span it), else
    // row-major
    const bool big = 2.0 * (double)M * (double)N * (double)K >= 4e9;
    const long long ldn = N + (N & 1);  // B's row stride on the k-major path: even, for 16-byte rows
    const bool kmajor = big && M >= 128 && N >= 128 && ((M + 127) / 128) * ((N + 127) / 128) >= 512 &&
                        ladder_t_min_chunks((int)K, M + (M & 1), ldn) >= 1;
    // A
    if (kmajor) {
        if (p.a == Kl + Ml && M % 2 == 0) { g.A = A; g.sAm = 1; g.sAk = M; }
        else {
            const long long ldm = M + (M & 1);  // even, for 16-byte rows
            double* t = ws.take<double>(K * ldm);
            if (ldm == M) {
                permute_any(t, A, p.a, adims, Kl + Ml, 1.0, 0.0, s);
            } else {
                double* u = ws.take<double>(K * M);
                permute_any(u, A, p.a, adims, Kl + Ml, 1.0, 0.0, s);
                k_copy2d(t, ldm, u, M, K, M, 1.0, 0.0, s);
            }
            g.A = t; g.sAm = 1; g.sAk = ldm;
        }
    } else if (p.a == Ml + Kl) { g.A = A; g.sAm = K; g.sAk = 1; }
    else if (p.a == Kl + Ml && !big) { g.A = A; g.sAm = 1; g.sAk = M; }
    else {
        double* t = ws.take<double>(M * K);
        permute_any(t, A, p.a, adims, Ml + Kl, 1.0, 0.0, s);
        g.A = t; g.sAm = K; g.sAk = 1;
    }
    // B
    if (kmajor && !(p.b == Kl + Nl && ldn == N && ((uintptr_t)B & 15) == 0)) {
        // [K][N] with an even row stride
        double* t = ws.take<double>(K * ldn);
        if (ldn == N) {
            permute_any(t, B, p.b, bdims, Kl + Nl, 1.0, 0.0, s);
        } else {
            double* u = ws.take<double>(K * N);
            permute_any(u, B, p.b, bdims, Kl + Nl, 1.0, 0.0, s);
            k_copy2d(t, ldn, u, N, K, N, 1.0, 0.0, s);
        }
        g.B = t; g.sBk = ldn; g.sBn = 1;
    } else if (p.b == Kl + Nl) { g.B = B; g.sBk = N; g.sBn = 1; }
    else if (p.b == Nl + Kl && !big) { g.B = B; g.sBk = 1; g.sBn = K; }
    else {
        double* t = ws.take<double>(K * N);
        permute_any(t, B, p.b, bdims, Kl + Nl, 1.0, 0.0, s);
        g.B = t; g.sBk = N; g.sBn = 1;
    }
    // C
    if (p.o == Ml + Nl) { g.C = C; g.sCm = N; g.sCn = 1; g.beta = beta; gemm(g, s); }
    else if (p.o == Nl + Ml && !big) { g.C = C; g.sCm = 1; g.sCn = M; g.beta = beta; gemm(g, s); }
    else {
        double* t = ws.take<double>(M * N);
        g.C = t; g.sCm = N; g.sCn = 1; g.beta = 0.0;
        gemm(g, s);
        int tdims[4];
        std::string tl = Ml + Nl;
        for (size_t k = 0; k < tl.size(); ++k) tdims[k] = odims[p.o.find(tl[k])];
        permute_any(C, t, tl, tdims, p.o, 1.0, beta, s);
    }
    ws.release(mark);
}

}  // namespace adc3
