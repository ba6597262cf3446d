// EA-ADC(2)/ADC(3) secular matrix, sigma build, Davidson and the SS-FNO/NAF pipeline.
//
// Closed-shell, density-fitted (eq 25): integrals with at most two virtual indices
// are formed once ((ia|jb), (ij|ab)); three-virtual integrals only enter the
// one-time 1p/2p1h coupling build.  The ladder term sum_cd (ac|bd) z_cd takes one of
// two forms: stored, where (ac|bd) is assembled once per basis from the DF factor on
// the matrix cores and kept in HBM as its pair-symmetric and pair-antisymmetric
// blocks G+ [(a<=b)][(c<=d)] and G- [(a<b)][(c<d)] (about v^4/2 doubles: 6.4 GB at
// v = 200), so a ladder application is two products against G+ and G- between a pack
// and an unpack of z; or assembled, sum_Q B^Q z B^Q from the factor in every
// application, when the stored blocks would exceed 96 GB in FP64 (v > 393).
//
// Vector layout: r = [r1[v], z[o][v][v]], z orthonormal doublet coordinates;
// x = z_S + z_A/sqrt(3) are the alpha-beta determinant coefficients and
// sigma_z = S(sigma_D) + sqrt(3) A(sigma_D).
//
// Secular matrix blocks (Sec. "Algebraic Diagrammatic Construction (ADC) Theory",
// eq 5 truncated; closed forms derived from the intermediate-state definition):
//   M11 = diag(e_v) - sym(P[T])                                  (through 2nd order)
//        + static self-energy of the 2nd-order density - sym(P[U2])
//        - sym(sum T (2L - L~)) - sym(ring)                       (3rd order, ADC(3))
//   U_D[a,b,c,i] = (ab|ic) + (2nd-order terms, ADC(3))
//   K  = e_a + e_b - e_i + (ladder + particle-hole terms, ADC(3))
// with T the first-order amplitudes T^ab_ij = (ia|jb)/(e_i+e_j-e_a-e_b),
// P[A]_ab = sum_klc (2A^ac_kl - A^ca_kl)(kb|lc), L^ab_ij = sum_cd (ac|bd) T^cd_ij.
#include "internal.h"
#include "tensor.h"
#include "../../include/adc3ea.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <exception>
#include <thread>
#include <vector>

namespace adc3 {

namespace {
thread_local std::string g_msg;
}

void set_error(const std::string& msg) { g_msg = msg; }
[[noreturn]] void fail(int status, const std::string& msg) { throw Error{status, msg}; }

// ADC3_VERBOSE=1 in the environment prints one line per pipeline phase to stderr
static int verbosity() {
    static const int v = [] {
        const char* e = std::getenv("ADC3_VERBOSE");
        return (e && e[0] >= '1' && e[0] <= '9') ? e[0] - '0' : 0;
    }();
    return g_dry ? 0 : v;
}
static bool verbose() { return verbosity() >= 1; }
#define VLOG(...)                                 \
    do {                                          \
        if (verbose()) {                          \
            std::fprintf(stderr, "[adc3] " __VA_ARGS__); \
            std::fprintf(stderr, "\n");           \
            std::fflush(stderr);                  \
        }                                         \
    } while (0)

// Small read-backs go through a pinned staging buffer (one per host thread, freed when the thread
// ends): the Davidson loop reads back a few numbers several times per iteration, and a copy into
// pageable memory is staged by the runtime at a higher latency.
namespace {
struct PinnedStage {
    void* p = nullptr;
    ~PinnedStage() {
        if (p) (void)hipHostFree(p);
    }
};
}  // namespace
static void d2h(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (g_dry) {
        std::memset(dst, 0, bytes);
        return;
    }
    constexpr size_t PIN = 1 << 20;
    thread_local PinnedStage pin;
    if (bytes <= PIN) {
        if (!pin.p) HIPCHK(hipHostMalloc(&pin.p, PIN, hipHostMallocDefault));
        HIPCHK(hipMemcpyAsync(pin.p, src, bytes, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::memcpy(dst, pin.p, bytes);
        return;
    }
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}
static void h2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (g_dry) return;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
constexpr int NVMAX = 16;  // vectors per sigma pass
// MI355X published peaks (dense matrix-core rates; HBM3E bandwidth), for roofline bounds
constexpr double PEAK_FP64_MFMA = 78.6e12, PEAK_FP32_MFMA = 157.3e12, PEAK_BF16_MFMA = 2.5e15, PEAK_HBM = 8.0e12;

struct Ctx {
    int o = 0, v = 0, X = 0, level = 2;
    double smx = 1.0;  // level 3: M = M_ADC(2) + smx (M_ADC(3) - M_ADC(2)) (scaled third order; 1 = ADC(3))
    long long N = 0;
    Arena ws;
    double *eo = nullptr, *ev = nullptr, *Boo = nullptr, *Bov = nullptr, *Bvv = nullptr;
    double *ovov = nullptr, *oovv = nullptr, *T = nullptr, *M11 = nullptr, *Uz = nullptr, *diag = nullptr;
    double *Dmp2 = nullptr;
    double *u1 = nullptr;  // second-order singles [o][v]: static self-energy and spectral amplitudes
    // eigendecomposition of M11 for the block preconditioner (computed on first use)
    double *m11_Q = nullptr, *m11_w = nullptr, *m11_tmp = nullptr;
    bool m11_eig = false;
    // stored ladder (level 3): the pair-symmetric block G+ [sa_lp(v)]^2 followed by the antisymmetric
    // block G- [sa_lm(v)]^2 (Gm points at it)
    double *G = nullptr, *Gm = nullptr;
    bool df = false;          // ladder assembled from Bvv in every application instead of stored
    double *P1 = nullptr;     // (ij|bd) as [i][b][j][d], level 3
    double *zb = nullptr, *xb = nullptr, *xtb = nullptr, *sdb = nullptr, *sb = nullptr;
    long long sigma_count = 0;
    // reduced-precision copies (precision 1: FP32 ladder and coupling; 2: BF16 ladder, FP32 coupling)
    int prec = 0;
    void* Glo = nullptr;    // reduced-precision G+ followed by G-
    void* Gmlo = nullptr;
    void* Bvvlo = nullptr;  // reduced-precision Bvv for the assembled ladder
    float* Bvv32 = nullptr; // BF16 contexts with the assembled ladder: an FP32 Bvv as well (middle phase)
    void* zlo = nullptr;  // reduced-precision copy of the ladder's input rows
    float* Uz32 = nullptr;
    // learned preconditioner: weights (caller's device memory) and the BF16 W2 copy
    const float* mlp_w = nullptr;
    unsigned short* mlp_wb = nullptr;
    // sigma temporaries live in a region fixed for the context's lifetime, so a sigma pass
    // captured into a HIP graph stays valid; gin/gout stage the vectors of a replayed pass
    char* sig_base = nullptr;
    size_t sig_bytes = 0;
    double *gin = nullptr, *gout = nullptr;
    bool graphs = false;
    std::map<int, hipGraphExec_t> graph_exec;  // key: vectors * 4 + precision
    ~Ctx() {
        for (auto& kv : graph_exec) (void)hipGraphExecDestroy(kv.second);
    }
};

static double* take(Arena& ws, long long n) { return ws.take<double>((size_t)std::max<long long>(n, 1)); }
// stand-in vectors of the counting dry runs (never dereferenced: no work is issued in a dry run)
static double* dry_vec() { return reinterpret_cast<double*>(ARENA_COUNT_BASE); }

// The ladder is assembled from Bvv in each application (instead of stored) when the stored blocks
// (about v^4 / 2 elements) would not leave room for the rest: above 96 GB in FP64 (v > 393).
static long long stored_ladder_elems(int v) { return sa_lp(v) * sa_lp(v) + sa_lm(v) * sa_lm(v); }
static bool ladder_df_auto(int v) { return (double)stored_ladder_elems(v) * 8.0 > 96e9; }
// Element budget of one chunk of the large setup tensors (o*na*v^2 per tensor of the coupling build);
// the assembled ladder's intermediate gets twice this.
static std::atomic<long long> g_chunk_elems{1LL << 29};
// Elements of the assembled ladder's intermediate for M rows: all X auxiliary functions at once when
// that fits the budget, else chunks of them (at least one).
static long long df_v_elems(int M, int v, int X) {
    const long long per = (long long)M * v * v;
    return std::max<long long>(1, std::min<long long>((long long)std::max(X, 1) * per, std::max<long long>(per, 2 * g_chunk_elems.load())));
}
static void sigma_pass(Ctx* c, Arena& ws, const double* rr, double* ss, int nv, hipStream_t s, int prec);
static size_t sigma_region_bytes(Ctx* c);

// symmetric part, scaled: M += a * (P + P^T)/2, P destroyed
static void add_sym(double* M, double* P, int v, double a, hipStream_t s) {
    k_symmetrize(P, v, s);
    k_axpby(M, P, (long long)v * v, a, 1.0, s);
}

// Build the context from DF blocks (copied in).  Temporaries are released on return.
static Ctx* build_ctx(Arena& ws, const double* eo_in, const double* ev_in, const double* Boo_in, const double* Bov_in,
                      const double* Bvv_in, int o, int v, int X, int level, hipStream_t s, int prec = 0,
                      bool df = false, double smx = 1.0) {
    ProfScope prof(PROF_SETUP, s, 0.0, 0.0);
    Ctx* c = new Ctx();
    c->o = o; c->v = v; c->X = X; c->level = level; c->prec = prec;
    c->smx = level >= 3 ? smx : 1.0;
    c->df = df && level >= 3;
    c->N = v + (long long)o * v * v;
    const long long oo = (long long)o * o, ov = (long long)o * v, vv = (long long)v * v;
    c->eo = take(ws, o); c->ev = take(ws, v);
    k_copy(c->eo, eo_in, o, s);
    k_copy(c->ev, ev_in, v, s);
    c->Boo = take(ws, X * oo); c->Bov = take(ws, X * ov); c->Bvv = take(ws, X * vv);
    k_copy(c->Boo, Boo_in, X * oo, s);
    k_copy(c->Bov, Bov_in, X * ov, s);
    k_copy(c->Bvv, Bvv_in, X * vv, s);
    const double *Boo = c->Boo, *Bov = c->Bov, *Bvv = c->Bvv, *eo = c->eo, *ev = c->ev;

    c->ovov = take(ws, ov * ov);
    ein(ws, "Qia,Qjb->iajb", 1.0, TV(Bov, {X, o, v}), TV(Bov, {X, o, v}), 0.0, c->ovov, s);
    c->oovv = take(ws, oo * vv);
    ein(ws, "Qij,Qab->ijab", 1.0, TV(Boo, {X, o, o}), TV(Bvv, {X, v, v}), 0.0, c->oovv, s);
    c->T = take(ws, oo * vv);
    k_amp_t(c->ovov, eo, ev, o, v, c->T, s);
    const double* T = c->T;
    c->M11 = take(ws, vv);
    c->m11_Q = take(ws, vv);
    c->m11_w = take(ws, v);
    c->m11_tmp = take(ws, vv + (long long)eig_large_scratch(v) + v);
    c->Dmp2 = take(ws, vv);
    c->u1 = take(ws, ov);
    c->diag = take(ws, c->N);
    c->Uz = take(ws, v * (long long)o * vv);
    if (level >= 3) {
        c->P1 = take(ws, oo * vv);
    }
    if (prec > 0) {
        c->Uz32 = ws.take<float>((size_t)std::max<long long>(v * (long long)o * vv, 1));
        if (level >= 3) {
            const long long ng = c->df ? std::max<long long>((long long)X * vv, 1) : stored_ladder_elems(v);
            void*& lo = c->df ? c->Bvvlo : c->Glo;
            if (prec == 1) lo = ws.take<float>((size_t)ng);
            else lo = ws.take<unsigned short>((size_t)ng);
            if (!c->df && lo) c->Gmlo = (char*)lo + sa_lp(v) * sa_lp(v) * (prec == 1 ? 4 : 2);
            if (prec == 2 && c->df) c->Bvv32 = ws.take<float>((size_t)ng);
            // the ladder's input rows: v^2 elements (assembled) or the two packed blocks (stored)
            c->zlo = ws.take<float>((size_t)(NVMAX * (long long)o * (sa_lp(v) + sa_lm(v))));
        }
    }
    c->mlp_wb = ws.take<unsigned short>(256 * 256);
    c->zb = take(ws, NVMAX * (long long)o * vv);
    // xb, xtb, sdb are contiguous: before the particle-hole terms use them they hold the
    // ladder's split-K partial sums
    c->xb = take(ws, 3 * NVMAX * (long long)o * vv);
    c->xtb = c->xb + NVMAX * (long long)o * vv;
    c->sdb = c->xtb + NVMAX * (long long)o * vv;
    c->sb = take(ws, NVMAX * (long long)o * vv);
    c->gin = take(ws, NVMAX * c->N);
    c->gout = take(ws, NVMAX * c->N);
    c->sig_bytes = sigma_region_bytes(c);
    c->sig_base = ws.take<char>(c->sig_bytes);
    // ---- temporaries below; G is taken only after the U_D phase has released its own, so the
    // setup peak is G plus the larger phase rather than G plus both ----
    const size_t mark0 = ws.mark();
    {
        // phase A: D^MP2, M11 through second order, U_D (first and second order) -> U_z
        GemmScratch gscr(ws, GEMM_SCRATCH);
        double* Tt2 = take(ws, oo * vv);  // 2T - T~
        k_comb_t(Tt2, T, oo, v, 2.0, -1.0, s);
        // MP2 virtual density (per spin): sum_klc (2T^ce_kl - T^ec_kl) T^cd_kl
        ein(ws, "klce,klcd->ed", 1.0, TV(Tt2, {o, o, v, v}), TV(T, {o, o, v, v}), 0.0, c->Dmp2, s);
        // M11 through second order
        double* P = take(ws, vv);
        ein(ws, "klac,kblc->ab", 1.0, TV(Tt2, {o, o, v, v}), TV(c->ovov, {o, v, o, v}), 0.0, P, s);
        k_fill(c->M11, vv, 0.0, s);
        add_sym(c->M11, P, v, -1.0, s);
        k_add_diag(c->M11, ev, v, s);
        if (level >= 3) {
            // permuted integrals for the particle-hole sigma terms
            int d_oovv[4] = {o, o, v, v};
            int p1[4] = {0, 2, 1, 3};  // [i][j][b][d] -> [i][b][j][d]
            k_permute4(c->P1, c->oovv, d_oovv, p1, 1.0, 0.0, s);
        }
        double* ooov = take(ws, oo * ov);
        ein(ws, "Qij,Qka->ijka", 1.0, TV(Boo, {X, o, o}), TV(Bov, {X, o, v}), 0.0, ooov, s);
        // W^Q_ic = sum_kd B^Q_kd (2T-T~)_ik^cd, and the second-order singles
        // u1_ia = [sum_Qc B^Q_ac W^Q_ic - sum_klc (2T-T~)_kl^ac (ki|lc)] / (e_i - e_a)
        double* Bw = take(ws, X * ov);
        ein(ws, "Qkd,ikcd->Qic", 1.0, TV(Bov, {X, o, v}), TV(Tt2, {o, o, v, v}), 0.0, Bw, s);
        ein(ws, "Qac,Qic->ia", 1.0, TV(Bvv, {X, v, v}), TV(Bw, {X, o, v}), 0.0, c->u1, s);
        ein(ws, "klac,kilc->ia", -1.0, TV(Tt2, {o, o, v, v}), TV(ooov, {o, o, o, v}), 1.0, c->u1, s);
        k_div_d1(c->u1, eo, ev, o, v, s);
        // U_D[a][b][c][i] (first order (ab|ic), second order below) and U_z[a][i][b][c] = S + sqrt3 A over
        // (b,c), in chunks of the first virtual index a when the o v^3 tensors would crowd HBM (each
        // chunk holds a few tensors of o*na*v^2 elements)
        const int na = (int)std::max<long long>(1, std::min<long long>(v, g_chunk_elems.load() / std::max<long long>(o * vv, 1)));
        double *Bvc = nullptr, *Boc = nullptr, *ooc = nullptr;
        if (na < v) {
            Bvc = take(ws, (long long)X * na * v);
            if (level >= 3) {
                Boc = take(ws, (long long)X * o * na);
                ooc = take(ws, oo * o * na);
            }
        }
        // second-order coupling term sum_kd (2T-T~)_ik^cd (kd|ab) = sum_Q B^Q_ab W^Q_ic, W^Q_ic = sum_kd B^Q_kd
        // (2T-T~)_ik^cd: folded into the first-order product as B^Q_ab (B^Q_ic + W^Q_ic)
        const double* Bov_u = Bov;
        if (level >= 3) {
            k_axpby(Bw, Bov, X * ov, 1.0, c->smx, s);  // B + smx W (second order scaled for sm-ADC)
            Bov_u = Bw;
        }
        k_fill(c->Uz, vv * ov, 0.0, s);
        for (int a0 = 0; a0 < v; a0 += na) {
            const int nc = std::min(na, v - a0);
            const size_t mchunk = ws.mark();
            const long long E = (long long)nc * v * v * o;
            // the chunk's slices of Bvv [X][a][b] and Bov [X][k][a]
            const double* Bvv_a = Bvv;
            if (na < v) {
                k_copy2d(Bvc, (long long)nc * v, Bvv + (long long)a0 * v, vv, X, (long long)nc * v, 1.0, 0.0, s);
                Bvv_a = Bvc;
            }
            double* Ud = take(ws, E);
            ein(ws, "Qab,Qic->abci", 1.0, TV(Bvv_a, {X, nc, v}), TV(Bov_u, {X, o, v}), 0.0, Ud, s);
            if (level >= 3) {
                TV tT(T, {o, o, v, v});
                const double *ooov_a = ooov, *Bov_a = Bov;
                if (na < v) {
                    k_copy2d(ooc, nc, ooov + a0, v, oo * o, nc, 1.0, 0.0, s);
                    k_copy2d(Boc, nc, Bov + a0, v, (long long)X * o, nc, 1.0, 0.0, s);
                    ooov_a = ooc;
                    Bov_a = Boc;
                }
                // coupling, second order (scaled by smx for sm-ADC)
                const double x2 = c->smx;
                ein(ws, "klbc,ilka->abci", x2, tT, TV(ooov_a, {o, o, o, nc}), 1.0, Ud, s);
                // (ka|cd) for a in the chunk: [k][a][c][d]
                double* ovvv1 = take(ws, E);
                ein(ws, "Qka,Qcd->kacd", 1.0, TV(Bov_a, {X, o, nc}), TV(Bvv, {X, v, v}), 0.0, ovvv1, s);
                TV t1(ovvv1, {o, nc, v, v});
                ein(ws, "kibd,kacd->abci", -x2, tT, t1, 1.0, Ud, s);
                ein(ws, "ikcd,kabd->abci", -x2, tT, t1, 1.0, Ud, s);
            }
            double* Up = take(ws, E);
            int d[4] = {nc, v, v, o}, pm[4] = {0, 3, 1, 2};
            k_permute4(Up, Ud, d, pm, 1.0, 0.0, s);
            k_d_to_z_add(c->Uz + (long long)a0 * o * vv, Up, (long long)nc * o, v, s);
            ws.release(mchunk);
        }
    }
    ws.release(mark0);
    if (level >= 3) {
        if (!c->df) {
            c->G = take(ws, stored_ladder_elems(v));  // kept with the context
            c->Gm = c->G + sa_lp(v) * sa_lp(v);
        }
        const size_t mark1 = ws.mark();
        // sm-ADC: M11 through second order, kept to scale the third-order part afterwards
        double* M11_2 = nullptr;
        if (c->smx != 1.0) {
            M11_2 = take(ws, vv);
            k_copy(M11_2, c->M11, vv, s);
        }
        {
            // phase B: G, then everything of M11 through third order that needs it
            GemmScratch gscr(ws, GEMM_SCRATCH);
            double* Tt2 = take(ws, oo * vv);
            k_comb_t(Tt2, T, oo, v, 2.0, -1.0, s);
            double* P = take(ws, vv);
            // stored ladder: for a chunk of a, (ac|bd) = sum_Q B^Q_ac B^Q_bd as one GEMM with rows (a,c) (from a
            // transposed copy of Bvv) and columns (b,d), b from the chunk's first a, then folded into the pair
            // blocks G+ and G-
            if (!c->df) {
                const long long v3 = (long long)v * vv;
                // chunk: at most an eighth of the stored blocks (and the chunk budget)
                const long long budget = std::min<long long>(g_chunk_elems.load(), stored_ladder_elems(v) / 8);
                const int na = (int)std::max<long long>(
                    1, std::min<long long>({(long long)v, budget / std::max<long long>(v3, 1), 65535 / v}));
                const size_t mg = ws.mark();
                double* Gf = take(ws, (long long)na * v3);
                double* BT = take(ws, vv * X);  // [(a,c)][Q]
                {
                    int d4[4] = {1, X, v, v}, p4[4] = {0, 2, 3, 1};
                    k_permute4(BT, Bvv, d4, p4, 1.0, 0.0, s);
                }
                for (int a0 = 0; a0 < v; a0 += na) {
                    const int nc = std::min(na, v - a0);
                    const long long ldf = (long long)(v - a0) * v;
                    gemm_rm(nc * v, (int)ldf, X, 1.0, BT + (long long)a0 * v * X, X, false, Bvv + (long long)a0 * v, vv,
                            false, 0.0, Gf, ldf, s);
                    k_sa_form(Gf, ldf, a0, nc, v, c->G, c->Gm, s);
                }
                k_sa_zero_pad_rows(c->G, c->Gm, v, s);
                ws.release(mg);
            }
            double* oooo = take(ws, oo * oo);
            ein(ws, "Qij,Qkl->ijkl", 1.0, TV(Boo, {X, o, o}), TV(Boo, {X, o, o}), 0.0, oooo, s);
            double* ooov = take(ws, oo * ov);
            ein(ws, "Qij,Qka->ijka", 1.0, TV(Boo, {X, o, o}), TV(Bov, {X, o, v}), 0.0, ooov, s);
            // second-order doubles residual Y (alpha-beta block)
            double* L = take(ws, oo * vv);
            if (c->df) {
                // T^cd_ij = T^dc_ji, so L_ji = L_ij^T: only the pairs i <= j are contracted
                const long long np = oo / 2 + o / 2 + (o % 2);  // o(o+1)/2
                const long long ve = df_v_elems((int)np, v, X);
                double* Vt = take(ws, ve);
                double* pr = take(ws, 2 * np * vv);
                df_ladder_pairs(o, v, X, Bvv, T, L, pr, Vt, ve, s);
            } else {
                // through the pair blocks, for the occupied pairs i <= j only (L_ji = L_ij^T):
                // L = unpack(G+ w+(T), G- w-(T))
                const long long lp = sa_lp(v), lm = sa_lm(v), np = (long long)o * (o + 1) / 2;
                double* Tp = take(ws, np * vv);
                double* Lp = take(ws, np * vv);
                double* W = take(ws, np * (lp + lm));
                double* CW = take(ws, np * (lp + lm));
                k_pairs_gather(Tp, T, o, v, s);
                k_sa_pack(Tp, vv, (int)np, v, W, W + np * lp, s);
                // the packed rows k-major for the ladder kernel that copies both tiles into LDS (K split
                // into 8 chunks, partial sums here), else the GEMM
                const long long ldt = (np + 1) / 2 * 2;
                double* Wt = take(ws, ldt * (lp + lm));
                double* part = take(ws, 8 * np * lp);
                k_transpose(W, lp, (int)np, lp, Wt, ldt, s);
                if (lm > 0) k_transpose(W + np * lp, lm, (int)np, lm, Wt + ldt * lp, ldt, s);
                for (int blk = 0; blk < 2; ++blk) {
                    const long long n = blk == 0 ? lp : lm;
                    if (n == 0) continue;
                    const double* Gb = blk == 0 ? c->G : c->Gm;
                    const double* Zt = Wt + (blk == 0 ? 0 : ldt * lp);
                    double* C = CW + (blk == 0 ? 0 : np * lp);
                    if (!(ladder_t_supported((int)np, (int)n, (int)n, Zt, ldt, Gb, n) &&
                          ladder_gemm_t((int)np, (int)n, (int)n, 1.0, Zt, ldt, Gb, n, 0.0, C, n, 8, part, 8 * np * lp, s,
                                        2)))
                        gemm_rm((int)np, (int)n, (int)n, 1.0, W + (blk == 0 ? 0 : np * lp), n, false, Gb, n, false, 0.0,
                                C, n, s);
                }
                k_sa_unpack(CW, CW + np * lp, (int)np, v, Lp, vv, s);
                k_pairs_scatter(L, Lp, o, v, s);
            }
            double* Y = take(ws, oo * vv);
            k_copy(Y, L, oo * vv, s);
            TV tT(T, {o, o, v, v}), tT2(Tt2, {o, o, v, v}), tovov(c->ovov, {o, v, o, v}), toovv(c->oovv, {o, o, v, v});
            ein(ws, "klab,kilj->ijab", 1.0, tT, TV(oooo, {o, o, o, o}), 1.0, Y, s);
            ein(ws, "ikac,jbkc->ijab", 1.0, tT2, tovov, 1.0, Y, s);
            ein(ws, "ikac,kjbc->ijab", -1.0, tT, toovv, 1.0, Y, s);
            ein(ws, "kjac,kibc->ijab", -1.0, tT, toovv, 1.0, Y, s);
            ein(ws, "ikcb,kjac->ijab", -1.0, tT, toovv, 1.0, Y, s);
            ein(ws, "jkbc,iakc->ijab", 1.0, tT2, tovov, 1.0, Y, s);
            ein(ws, "jkbc,kiac->ijab", -1.0, tT, toovv, 1.0, Y, s);
            double* U2 = Y;  // in place: U2 = Y / D
            k_div_d2(U2, eo, ev, o, v, s);
            const double* u1 = c->u1;  // second-order singles (formed with the coupling)
            // second-order densities (per spin)
            double* roo = take(ws, oo);
            ein(ws, "mkcd,lkcd->ml", -1.0, tT2, tT, 0.0, roo, s);
            const double* rvv = c->Dmp2;
            // static self-energy  sum_pq <ap||bq> rho_pq
            double* J = take(ws, X);
            gemm_rm(X, 1, (int)oo, 1.0, Boo, oo, false, roo, 1, false, 0.0, J, 1, s);
            gemm_rm(X, 1, (int)vv, 1.0, Bvv, vv, false, rvv, 1, false, 1.0, J, 1, s);
            gemm_rm(X, 1, (int)ov, 2.0, Bov, ov, false, u1, 1, false, 1.0, J, 1, s);
            gemm_rm((int)vv, 1, X, 2.0, Bvv, vv, true, J, 1, false, 1.0, c->M11, 1, s);
            double* Z1 = take(ws, X * ov);
            ein(ws, "ml,Qlb->Qmb", 1.0, TV(roo, {o, o}), TV(Bov, {X, o, v}), 0.0, Z1, s);
            ein(ws, "Qma,Qmb->ab", -1.0, TV(Bov, {X, o, v}), TV(Z1, {X, o, v}), 1.0, c->M11, s);
            double* Z2 = take(ws, X * vv);
            ein(ws, "Qad,ed->Qae", 1.0, TV(Bvv, {X, v, v}), TV(rvv, {v, v}), 0.0, Z2, s);
            ein(ws, "Qae,Qeb->ab", -1.0, TV(Z2, {X, v, v}), TV(Bvv, {X, v, v}), 1.0, c->M11, s);
            double* Z3 = Z1;
            ein(ws, "Qbc,kc->Qkb", 1.0, TV(Bvv, {X, v, v}), TV(u1, {o, v}), 0.0, Z3, s);
            ein(ws, "Qka,Qkb->ab", -1.0, TV(Bov, {X, o, v}), TV(Z3, {X, o, v}), 1.0, c->M11, s);
            ein(ws, "Qkb,Qka->ab", -1.0, TV(Bov, {X, o, v}), TV(Z3, {X, o, v}), 1.0, c->M11, s);
            // second-order form with second-order amplitudes
            double* U2t2 = take(ws, oo * vv);
            k_comb_t(U2t2, U2, oo, v, 2.0, -1.0, s);
            ein(ws, "klac,kblc->ab", 1.0, TV(U2t2, {o, o, v, v}), tovov, 0.0, P, s);
            add_sym(c->M11, P, v, -1.0, s);
            // ladder part: - sym( sum_ekl T^ae_kl (2 L^be_kl - L^eb_kl) )
            double* Lt2 = U2t2;
            k_comb_t(Lt2, L, oo, v, 2.0, -1.0, s);
            ein(ws, "klae,klbe->ab", 1.0, tT, TV(Lt2, {o, o, v, v}), 0.0, P, s);
            add_sym(c->M11, P, v, -1.0, s);
            // ring part
            double* g1 = take(ws, oo * vv);   // [d][l][b][m] = (db|ml) - (dl|mb)
            double* g2 = take(ws, oo * vv);   // [d][l][b][m] = (dl|mb)
            double* g3 = take(ws, oo * vv);   // [d][l][b][m] = (db|ml)
            {
                int d_oovv[4] = {o, o, v, v}, p_oovv[4] = {2, 1, 3, 0};  // oovv[m][l][d][b] -> [d][l][b][m]
                int d_ovov[4] = {o, v, o, v}, p_ovov[4] = {1, 0, 3, 2};  // ovov[l][d][m][b] -> [d][l][b][m]
                k_permute4(g3, c->oovv, d_oovv, p_oovv, 1.0, 0.0, s);
                k_permute4(g2, c->ovov, d_ovov, p_ovov, 1.0, 0.0, s);
                k_copy(g1, g3, oo * vv, s);
                k_axpby(g1, g2, oo * vv, -1.0, 1.0, s);
            }
            double* TmT = Lt2;  // T - T~
            k_comb_t(TmT, T, oo, v, 1.0, -1.0, s);
            TV tg1(g1, {v, o, v, o}), tg2(g2, {v, o, v, o}), tg3(g3, {v, o, v, o}), tTm(TmT, {o, o, v, v});
            double* RA = take(ws, oo * vv);
            double* RB = take(ws, oo * vv);
            double* RC = take(ws, oo * vv);
            ein(ws, "klcd,dlbm->ckbm", 1.0, tTm, tg1, 0.0, RA, s);
            ein(ws, "klcd,dlbm->ckbm", -1.0, tT, tg2, 1.0, RA, s);
            ein(ws, "klcd,dlbm->ckbm", 1.0, tT, tg1, 0.0, RB, s);
            ein(ws, "klcd,dlbm->ckbm", -1.0, tTm, tg2, 1.0, RB, s);
            ein(ws, "kldc,dlbm->ckbm", -1.0, tT, tg3, 0.0, RC, s);
            TV tRA(RA, {v, o, v, o}), tRB(RB, {v, o, v, o}), tRC(RC, {v, o, v, o});
            ein(ws, "kmac,ckbm->ab", 1.0, tTm, tRA, 0.0, P, s);
            ein(ws, "mkac,ckbm->ab", -1.0, tT, tRB, 1.0, P, s);
            ein(ws, "kmac,ckbm->ab", 1.0, tT, tRC, 1.0, P, s);
            add_sym(c->M11, P, v, -1.0, s);
        }
        if (M11_2) k_axpby(c->M11, M11_2, vv, 1.0 - c->smx, c->smx, s);  // M11_2 + smx (M11_3 - M11_2)
        ws.release(mark1);
    }
    k_diag_adc(c->diag, c->M11, eo, ev, Bvv, c->oovv, c->ovov, o, v, X, level, s, c->smx);
    if (prec > 0) {
        k_to_lowp(c->Uz32, c->Uz, v * (long long)o * vv, 1, s);
        if (level >= 3 && c->df) {
            k_to_lowp(c->Bvvlo, c->Bvv, (long long)X * vv, prec, s);
            if (c->Bvv32) k_to_lowp(c->Bvv32, c->Bvv, (long long)X * vv, 1, s);
        } else if (level >= 3) {
            k_to_lowp(c->Glo, c->G, stored_ladder_elems(v), prec, s);
        }
    }
    c->ws = ws;  // snapshot (base/cap/used) for later temporaries
    return c;
}

// sigma = M r for nvec vectors
// One pass of at most NVMAX vectors: ss[nv][N] = M rr[nv][N], temporaries from ws.
static void sigma_pass(Ctx* c, Arena& ws, const double* rr, double* ss, int nv, hipStream_t s, int prec) {
    GemmScratch gscr(ws, GEMM_SCRATCH);
    const int o = c->o, v = c->v;
    const long long N = c->N, vv = (long long)v * v, ovv = (long long)o * vv;
    {
        // 1p: M11 r1 + U_z z
        gemm_rm(nv, v, v, 1.0, rr, N, false, c->M11, v, true, 0.0, ss, N, s);
        if (prec > 0) {
            // the FP32 copy of U_z: both products in one stream over it when it fits the fused kernel (sums in
            // FP64), else the two reduced-precision GEMMs (FP32 sums)
            const long long pe1 = v <= 256 ? 768LL * nv * v : 0;
            double* part1 = pe1 > 0 ? take(ws, pe1) : nullptr;
            const long long nch = (g_dry || pe1 == 0)
                                      ? 0
                                      : couple_fused32(nv, v, ovv, c->Uz32, ovv, rr + v, N, rr, N, ss + v, N, part1, pe1, s);
            if (nch > 0) {
                splitk_reduce(part1, (int)nch, nv, v, 1.0, 1.0, ss, N, 1, s);
            } else {
                GemmLP g;
                g.M = nv; g.N = v; g.K = (int)ovv;
                g.A = rr + v; g.sAm = N; g.sAk = 1;
                g.B = c->Uz32; g.sBk = 1; g.sBn = ovv;
                g.C = ss; g.sCm = N; g.sCn = 1; g.beta = 1.0;
                gemm_lp(g, 1, s);
                GemmLP h;
                h.M = nv; h.N = (int)ovv; h.K = v;
                h.A = rr; h.sAm = N; h.sAk = 1;
                h.B = c->Uz32; h.sBk = ovv; h.sBn = 1;
                h.C = ss + v; h.sCm = N; h.sCn = 1;
                gemm_lp(h, 1, s);
            }
        } else {
            // both U_z products (1p: U_z z, 2p1h: U_z^T r1) in one stream over U_z when it fits the fused
            // kernel (v <= 256, aligned rows), else one stream each
            const long long pe1 = v <= 256 ? 768LL * nv * v : 0;
            double* part1 = pe1 > 0 ? take(ws, pe1) : nullptr;
            const long long nch =
                (g_dry || pe1 == 0) ? 0 : couple_fused(nv, v, ovv, c->Uz, ovv, rr + v, N, rr, N, ss + v, N, part1, pe1, s);
            if (nch > 0) {
                splitk_reduce(part1, (int)nch, nv, v, 1.0, 1.0, ss, N, 1, s);
            } else {
                gemm_rm(nv, v, (int)ovv, 1.0, rr + v, N, false, c->Uz, ovv, true, 1.0, ss, N, s);
                // 2p1h: U_z^T r1, a stream over U_z [a][(i,b,c)]: on the k-major ladder kernel with r1
                // transposed ([a][n], a few KB), else as a GEMM
                const long long ldr = (nv + 1) / 2 * 2;
                double* r1t = take(ws, (long long)v * ldr);
                const bool t = ovv <= 0x7fffffffLL && ladder_t_supported(nv, (int)ovv, v, r1t, ldr, c->Uz, ovv) &&
                               ladder_t_min_chunks(v, ldr, ovv) == 1;
                if (t) k_transpose(rr, N, nv, v, r1t, ldr, s);
                if (!(t && ladder_gemm_t(nv, (int)ovv, v, 1.0, r1t, ldr, c->Uz, ovv, 0.0, ss + v, N, 1, nullptr, 0, s, 2)))
                    gemm_rm(nv, (int)ovv, v, 1.0, rr, N, false, c->Uz, ovv, false, 0.0, ss + v, N, s);
            }
        }
        k_k0_add(ss + v, rr + v, c->eo, c->ev, o, v, nv, N, s);
        if (c->level >= 3) {
            double* zb = c->zb;
            k_copy2d(zb, ovv, rr + v, N, nv, ovv, 1.0, 0.0, s);
            // ladder: sum_cd (ac|bd) z_cd  (G symmetric)
            if (c->df) {
                // assembled from Bvv: 4 X M v^3 flops; the intermediate is written and read once (and its
                // region is reused by the particle-hole terms below)
                const size_t mk = ws.mark();
                const int M = nv * o, X = c->X;
                const long long ve = df_v_elems(M, v, X);
                const double eb = prec == 0 ? 8.0 : prec == 1 ? 4.0 : 2.0;
                const double fl = 4.0 * X * (double)M * v * (double)vv;
                const double by = eb * (2.0 * X * (double)M * vv + (double)X * vv + M * (double)vv) + 8.0 * M * (double)vv;
                const double pk = prec == 0 ? PEAK_FP64_MFMA : prec == 1 ? PEAK_FP32_MFMA : PEAK_BF16_MFMA;
                ProfScope p(prec > 0 ? PROF_LADDER_LP : PROF_LADDER, s, fl, by, 1e3 * std::max(fl / pk, by / PEAK_HBM));
                if (prec > 0) {
                    const long long vl = prec == 2 ? ve + (long long)M * vv + 8 : ve;  // BF16: + Z transposed
                    void* V = prec == 1 ? (void*)ws.take<float>((size_t)vl) : (void*)ws.take<unsigned short>((size_t)vl);
                    k_to_lowp(c->zlo, zb, (long long)M * vv, prec, s);
                    // FP32 sigma of a BF16 context (its middle phase) takes the FP32 copy of Bvv
                    const void* Bl = (prec == 1 && c->prec == 2) ? (const void*)c->Bvv32 : c->Bvvlo;
                    df_ladder(prec, M, v, X, Bl, c->zlo, c->sb, false, V, vl, s);
                } else {
                    double* V = take(ws, ve);
                    df_ladder(0, M, v, X, c->Bvv, zb, c->sb, false, V, ve, s);
                }
                ws.release(mk);
            } else {
                // stored ladder through its pair blocks: w+- = pack(z), C+- = w+- G+-, sigma_z = unpack(C+-);
                // one profiled launch per block
                const int M = nv * o;
                const long long lp = sa_lp(v), lm = sa_lm(v);
                const size_t mk = ws.mark();
                double* W = take(ws, (long long)M * (lp + lm));
                double* CW = take(ws, (long long)M * (lp + lm));
                const long long pe = 3 * NVMAX * (long long)o * vv;
                k_sa_pack(zb, vv, M, v, W, W + (long long)M * lp, s);
                if (prec > 0) k_to_lowp(c->zlo, W, (long long)M * (lp + lm), prec, s);
                // FP64 with >= 3 row blocks (33 rows and up): the packed rows k-major, for the kernel that copies both tiles
                // straight into LDS (below that the G stream bounds the product and the row-major kernel,
                // with more workgroups per CU, streams it faster)
                // (FP32: the same, converted to FP32, rows padded to a multiple of 4)
                const long long ldt = prec == 1 ? (M + 3) / 4 * 4 : (M + 1) / 2 * 2;
                double* Wt = prec <= 1 ? take(ws, ldt * (lp + lm)) : nullptr;
                float* Wt32 = prec == 1 ? (float*)take(ws, (ldt * (lp + lm) + 1) / 2) : nullptr;
                int ltm, lmt;
                ladder_rows(M, ltm, lmt);
                const bool kmajor = prec <= 1 && ltm >= 3;
                if (kmajor) {
                    k_transpose(W, lp, M, lp, Wt, ldt, s);
                    k_transpose(W + (long long)M * lp, lm, M, lm, Wt + ldt * lp, ldt, s);
                    if (prec == 1) k_to_lowp(Wt32, Wt, ldt * (lp + lm), 1, s);
                }
                const int eb = prec == 0 ? 8 : prec == 1 ? 4 : 2;
                const double pk = prec == 0 ? PEAK_FP64_MFMA : prec == 1 ? PEAK_FP32_MFMA : PEAK_BF16_MFMA;
                for (int blk = 0; blk < 2; ++blk) {
                    const long long n = blk == 0 ? lp : lm;
                    if (n == 0) continue;
                    const long long woff = blk == 0 ? 0 : (long long)M * lp;
                    double* C = CW + woff;
                    const double fl = 2.0 * M * (double)n * n;
                    const double by = eb * (double)n * n + (eb + 8.0) * M * (double)n;
                    ProfScope p(prec > 0 ? PROF_LADDER_LP : PROF_LADDER, s, fl, by,
                                1e3 * std::max(fl / pk, by / PEAK_HBM));
                    if (prec > 0) {
                        const void* Z = (const char*)c->zlo + woff * eb;
                        const void* Gl = blk == 0 ? c->Glo : c->Gmlo;
                        const float* Zt32 = kmajor && prec == 1 ? Wt32 + (blk == 0 ? 0 : ldt * lp) : nullptr;
                        if (Zt32 && ladder_t32_supported(M, (int)n, (int)n, Zt32, ldt, (const float*)Gl, n) &&
                            ladder_gemm_t32(M, (int)n, (int)n, 1.0, Zt32, ldt, (const float*)Gl, n, 0.0, C, n,
                                            ladder_tuned_chunks(4, M, (int)n, (int)n, Zt32, ldt, Gl, n, C, n, c->xb, pe, s),
                                            c->xb, pe, s)) {
                            // done on the k-major FP32 kernel
                        } else if (ladder_lp_supported(prec, M, (int)n, (int)n, Z, n, Gl, n, C, n)) {
                            const int nch = ladder_tuned_chunks(prec, M, (int)n, (int)n, Z, n, Gl, n, C, n, c->xb, pe, s);
                            ladder_gemm_lp(prec, M, (int)n, (int)n, 1.0, Z, n, Gl, n, 0.0, C, n, nch, c->xb, pe, s);
                        } else {
                            GemmLP g;
                            g.M = M; g.N = (int)n; g.K = (int)n;
                            g.A = W + woff; g.sAm = n; g.sAk = 1;
                            g.B = Gl; g.sBk = n; g.sBn = 1;
                            g.C = C; g.sCm = n; g.sCn = 1;
                            gemm_lp(g, prec, s, 1);
                        }
                    } else {
                        const double* Z = W + woff;
                        const double* Gb = blk == 0 ? c->G : c->Gm;
                        const double* Zt = kmajor ? Wt + (blk == 0 ? 0 : ldt * lp) : nullptr;
                        if (kmajor && ladder_t_supported(M, (int)n, (int)n, Zt, ldt, Gb, n) &&
                            ladder_gemm_t(M, (int)n, (int)n, 1.0, Zt, ldt, Gb, n, 0.0, C, n,
                                          ladder_tuned_chunks(3, M, (int)n, (int)n, Zt, ldt, Gb, n, C, n, c->xb, pe, s),
                                          c->xb, pe, s)) {
                            // done on the k-major kernel
                        } else if (ladder_supported(M, (int)n, (int)n, Z, n, Gb, n, C, n)) {
                            const int nch = ladder_tuned_chunks(0, M, (int)n, (int)n, Z, n, Gb, n, C, n, c->xb, pe, s);
                            ladder_gemm(M, (int)n, (int)n, 1.0, Z, n, Gb, n, 0.0, C, n, nch, c->xb, pe, s);
                        } else {
                            gemm_rm(M, (int)n, (int)n, 1.0, Z, n, false, Gb, n, false, 0.0, C, n, s, 1);
                        }
                    }
                }
                k_sa_unpack(CW, CW + (long long)M * lp, M, v, c->sb, vv, s);
                ws.release(mk);
            }
            // particle-hole terms on the alpha-beta determinants x (z = S + sqrt3 A of x per block):
            //   d[n][i][a][b] = sum_jd (ib|jd) xt[n][j][a][d] - (ij|bd) x[n][j][a][d] - (ij|ad) x[n][j][d][b]
            // with rows (n,a) and columns (i,b): the first product through the DF factor,
            // (Y1 B^T) B with B = Bov as [Q][(j,d)] (its contraction indices j,d sit in one factor), the other
            // two (both against the same symmetric [(j,d)][(i,b)] matrix P1 = (ij|bd)) as one GEMM over the
            // stacked rows [Y2; Y3] (the ladder tile streams P1 once per row tile); then
            // sigma_z += S(d) + sqrt3 A(d)
            {
                const int Mph = nv * v, ovi = o * v, X = c->X;
                double *Y1 = c->xb, *Y2 = c->xtb;
                double* Y3 = Y2 + (long long)Mph * ovi;  // stacked under Y2 (inside the xtb/sdb region)
                k_ph_prep(zb, Y1, Y2, Y3, nv, o, v, s);
                double* D = zb;  // z is not needed any more: the factor product goes here
                double* E = take(ws, 2 * NVMAX * (long long)o * vv);
                const long long pe = 2 * NVMAX * (long long)o * vv;
                double* part = take(ws, pe);
                double* Wq = take(ws, (long long)NVMAX * v * X);
                // [Y2; Y3] k-major for the ladder kernel that copies both tiles into LDS, else the row-major tile
                const long long ldy = 2LL * Mph;
                double* Yt = take(ws, (long long)ovi * 2 * NVMAX * v);
                const bool tk = ladder_t_supported(2 * Mph, ovi, ovi, Yt, ldy, c->P1, ovi) &&
                                ladder_t_min_chunks(ovi, ldy, ovi) == 1;
                if (tk) k_transpose(Y2, ovi, 2 * Mph, ovi, Yt, ldy, s);
                const bool lad = !tk && ladder_supported(2 * Mph, ovi, ovi, Y2, ovi, c->P1, ovi, E, ovi);
                const int nch = tk    ? ladder_tuned_chunks(3, 2 * Mph, ovi, ovi, Yt, ldy, c->P1, ovi, E, ovi, part, pe, s)
                                : lad ? ladder_tuned_chunks(0, 2 * Mph, ovi, ovi, Y2, ovi, c->P1, ovi, E, ovi, part, pe, s)
                                      : 1;
                {
                    Gemm g;  // Wq[(n,a)][Q] = sum_(j,d) Y1[(n,a)][(j,d)] Bov[Q][(j,d)]
                    g.M = Mph; g.N = X; g.K = ovi;
                    g.A = Y1; g.sAm = ovi; g.sAk = 1;
                    g.B = c->Bov; g.sBk = 1; g.sBn = ovi;
                    g.C = Wq; g.sCm = X; g.sCn = 1;
                    gemm_split(g, s);
                }
                gemm_rm(Mph, ovi, X, 1.0, Wq, X, false, c->Bov, ovi, false, 0.0, D, ovi, s);
                // (a fixed chunk count may not fit the partial buffer: clamped, as the row-major path does)
                const int ncht = (int)std::max<long long>(1, std::min<long long>(nch, pe / (2LL * Mph * ovi)));
                if (tk && ladder_gemm_t(2 * Mph, ovi, ovi, 1.0, Yt, ldy, c->P1, ovi, 0.0, E, ovi, ncht, part, pe, s, 2)) {
                    // done on the k-major kernel
                } else if (lad) {
                    ladder_gemm(2 * Mph, ovi, ovi, 1.0, Y2, ovi, c->P1, ovi, 0.0, E, ovi, nch, part, pe, s, 2);
                } else {
                    gemm_rm(2 * Mph, ovi, ovi, 1.0, Y2, ovi, false, c->P1, ovi, false, 0.0, E, ovi, s);
                }
                k_ph_fin(c->sb, D, E, E + (long long)Mph * ovi, nv, o, v, s);
            }
            // first-order 2p1h terms (ladder + particle-hole), scaled by smx for sm-ADC
            k_copy2d(ss + v, N, c->sb, ovv, nv, ovv, c->smx, 1.0, s);
        }
    }
}

// Bytes of the fixed sigma region: the peak of a pass of NVMAX vectors at either precision.
static size_t sigma_region_bytes(Ctx* c) {
    const bool was = g_dry;
    g_dry = true;
    size_t peak = 0;
    for (int p : {0, c->prec, c->Bvv32 ? 1 : 0}) {
        Arena count;
        sigma_pass(c, count, dry_vec(), dry_vec(), NVMAX, nullptr, p);
        peak = std::max(peak, count.peak);
    }
    g_dry = was;
    return peak + 4096;
}

// The context's fixed sigma region as an arena.
static Arena sigma_arena(const Ctx* c) {
    Arena a;
    a.base = c->sig_base;
    a.cap = c->sig_bytes;
    return a;
}

// sigma = M r for nvec vectors, in passes of NVMAX.  With graphs on (and a non-null
// stream) each pass shape is captured once, after one eager pass that also settles the
// ladder tuner, and replayed on staged copies of the vectors.
static void sigma_impl(Ctx* c, Arena& wsin, const double* r, double* sg, int nvec, hipStream_t s, int prec = 0) {
    (void)wsin;
    if (prec > c->prec) prec = c->prec;
    ProfScope prof(PROF_SIGMA, s, 0.0, 0.0);
    const long long N = c->N;
    const bool use_graph = c->graphs && s != nullptr && !g_dry;
    for (int n0 = 0; n0 < nvec; n0 += NVMAX) {
        const int nv = std::min(NVMAX, nvec - n0);
        const double* rr = r + (long long)n0 * N;
        double* ss = sg + (long long)n0 * N;
        Arena sw = sigma_arena(c);
        if (!use_graph) {
            sigma_pass(c, sw, rr, ss, nv, s, prec);
            continue;
        }
        const int key = nv * 4 + prec;
        auto it = c->graph_exec.find(key);
        if (it == c->graph_exec.end()) {
            sigma_pass(c, sw, rr, ss, nv, s, prec);  // eager, and the tuner's first look at this shape
            hipGraph_t gr = nullptr;
            Arena sw2 = sigma_arena(c);
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            sigma_pass(c, sw2, c->gin, c->gout, nv, s, prec);
            HIPCHK(hipStreamEndCapture(s, &gr));
            hipGraphExec_t ex = nullptr;
            HIPCHK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
            HIPCHK(hipGraphDestroy(gr));
            c->graph_exec[key] = ex;
            continue;
        }
        k_copy(c->gin, rr, (long long)nv * N, s);
        HIPCHK(hipGraphLaunch(it->second, s));
        k_copy(ss, c->gout, (long long)nv * N, s);
    }
    c->sigma_count += nvec;
}

// ---------------------------------------------------------------------------
// Davidson (FP64, device-resident subspace)
// ---------------------------------------------------------------------------
// Training-data recorder of a replayed Jacobi solve whose converged vectors xf are known.
struct Recorder {
    int S = 0, Gmax = 0, G = 0;
    unsigned long long seed = 0;
    const double* xf = nullptr;                        // converged vectors [nroots][N]
    double *F = nullptr, *A0 = nullptr, *D = nullptr;  // caller buffers [Gmax][S][6], [Gmax][S], [Gmax][S]
};

// Failure injection for tests of the error path (adc3_debug_inject_nan): the next Davidson that
// reaches this iteration writes NaN into the sigma vector of its first new direction, once.
static std::atomic<int> g_nan_at{0};

struct DavResult {
    std::vector<double> w, rn;
    std::vector<double> w_lowp;  // Ritz values when the reduced-precision phase ended
    int iters = 0, iters_lowp = 0;
    bool converged = false;
};

static DavResult davidson_impl(Ctx* c, Arena& ws, int nroots, double conv, int max_iter, int max_sub,
                               double* vec_out, hipStream_t s, int prec = 0, bool use_mlp = false,
                               Recorder* rec = nullptr, const double* guess = nullptr, int nguess_in = 0,
                               int pmode = 0) {
    const bool olsen = pmode == 2, block1p = pmode == 3;
    if (prec > c->prec) prec = c->prec;
    ProfScope prof(PROF_DAVIDSON, s, 0.0, 0.0);
    const long long N = c->N;
    if (nroots < 1 || nroots > N) fail(-1, "davidson: nroots out of range");
    if (nroots > 40) fail(-1, "davidson: at most 40 roots per solve");
    int mmax = max_sub > 0 ? max_sub : std::max(8 * nroots, 40);
    mmax = std::max(mmax, 2 * nroots + 1);
    mmax = (int)std::min<long long>(std::min(mmax, 96), N);
    const int nguess = (int)std::min<long long>(N, std::min(nroots + 4, mmax));
    const size_t mark = ws.mark();
    double* V = take(ws, (long long)mmax * N);
    double* S = take(ws, (long long)mmax * N);
    double* Xr = take(ws, (long long)nroots * N);
    double* AX = take(ws, (long long)nroots * N);
    double* R = take(ws, (long long)std::max(nroots, 1) * N);
    double* Gm = take(ws, (long long)mmax * mmax);
    double* Gf = take(ws, (long long)mmax * mmax);  // Gram V S^T, kept incrementally (row stride mmax)
    double* Gw = take(ws, (long long)mmax * mmax + mmax);
    double* ev = take(ws, mmax);
    double* Y = take(ws, (long long)mmax * mmax);
    double* th = take(ws, nroots);
    double* coef = take(ws, (long long)mmax * mmax);
    const int nkeep_max = std::max(nroots, std::min(2 * nroots + 2, mmax / 2));
    double* Vk = take(ws, (long long)nkeep_max * N);
    double* Sk = take(ws, (long long)nkeep_max * N);
    double* small = take(ws, 16);
    unsigned int* mflag = (unsigned int*)take(ws, (mmax + 1) / 2);  // one flag word per new direction
    double* part = take(ws, (long long)dots_partial_elems(mmax, mmax, N));
    DavResult res;
    res.w.assign(nroots, 0.0);
    res.rn.assign(nroots, 0.0);
    if (g_dry) {
        sigma_impl(c, ws, V, S, std::min(NVMAX, nguess), s, prec);  // count the sigma temporaries too
        ws.release(mark);
        return res;
    }
    // Block orthonormalisation of the rows Tn[0..nn) against V[0..m) and within the block:
    // unit rows, then (one CGS pass + Loewdin over the kept directions), repeated when the
    // smallest kept Gram eigenvalue after the pass is below 1/2 (some direction lost more than
    // ~30% of its length to V or to the block: the second pass restores orthogonality, as in
    // the "twice is enough" rule).  tmp holds nn rows.  Returns the number kept.
    auto orthonormalise = [&](double* Tn, int nn, int m, double* tmp) -> int {
        k_dots(Tn, N, nn, Tn, N, nn, N, Gw, nn, part, s);
        k_rscale_rows(Tn, nn, N, Gw, nn, s);
        int acc = nn;
        bool again = true;
        for (int round = 0; round < 3 && acc > 0 && again; ++round) {
            if (m > 0) {
                k_dots(V, N, m, Tn, N, acc, N, coef, acc, part, s);
                k_lincomb(Tn, N, acc, V, N, m, coef, acc, N, -1.0, 1.0, s);
            }
            // Loewdin within the block: T' = (U w^-1/2)^T T over the kept directions
            k_dots(Tn, N, acc, Tn, N, acc, N, Gm, acc, part, s);
            k_symmetrize(Gm, acc, s);
            eig_small(Gm, acc, ev, Y, s);
            k_sort_eig(ev, Y, acc, 1, Gw, Gw + acc, s);
            std::vector<double> hq(acc);
            d2h(hq.data(), ev, acc * sizeof(double), s);
            int keep = 0;
            for (int q = 0; q < acc; ++q) keep += (hq[q] > 1e-14 && std::isfinite(hq[q]));
            if (keep == 0) return 0;
            again = hq[keep - 1] < 0.5;  // strong cancellation: orthonormalise once more
            k_lowdin_coef(coef, Y, ev, acc, keep, s);
            k_lincomb(tmp, N, keep, Tn, N, acc, coef, keep, N, 1.0, 0.0, s);
            k_copy(Tn, tmp, (long long)keep * N, s);
            acc = keep;
        }
        return acc;
    };
    // guesses: the caller's vectors first (if any), then unit vectors on the lowest diagonal
    // entries (ties by index)
    const int ng = guess ? std::min(nguess_in, nguess) : 0;
    std::vector<double> hd(N);
    d2h(hd.data(), c->diag, N * sizeof(double), s);
    // the (nguess - ng) lowest (value, index) pairs, ascending: a bounded max-heap, O(N log k), gives the
    // same entries as a stable sort of all N by value
    const int kneed = nguess - ng;
    std::vector<long long> idx;
    if (kneed > 0) {
        std::vector<std::pair<double, long long>> heap;
        heap.reserve(kneed + 1);
        for (long long i = 0; i < N; ++i) {
            const std::pair<double, long long> e(hd[i], i);
            if ((int)heap.size() < kneed) {
                heap.push_back(e);
                std::push_heap(heap.begin(), heap.end());
            } else if (e < heap.front()) {
                std::pop_heap(heap.begin(), heap.end());
                heap.back() = e;
                std::push_heap(heap.begin(), heap.end());
            }
        }
        std::sort_heap(heap.begin(), heap.end());
        for (const auto& e : heap) idx.push_back(e.second);
    }
    k_fill(V, (long long)nguess * N, 0.0, s);
    if (ng > 0) k_copy(V, guess, (long long)ng * N, s);
    std::vector<double> one(1, 1.0);
    for (int k = 0; k < nguess - ng; ++k) h2d(V + (long long)(ng + k) * N + idx[k], one.data(), sizeof(double), s);
    int m = nguess;
    if (block1p && !c->m11_eig) {
        const long long vv = (long long)c->v * c->v;
        k_copy(c->m11_tmp, c->M11, vv, s);
        eig_large(c->m11_tmp, c->v, c->m11_w, c->m11_Q, c->m11_tmp + vv + c->v, s);
        c->m11_eig = true;
    }
    if (ng > 0) {
        m = orthonormalise(V, nguess, 0, S);
        if (m < nroots) fail(-4, "davidson: initial guesses are linearly dependent");
    }
    // phase > 0: reduced-precision sigma until its noise floor, then FP64 correction (a BF16 context with
    // an FP32 copy of the factor passes through FP32 on the way)
    int phase = prec;
    std::vector<double> lp_best(nroots, INFINITY);
    std::vector<int> lp_stall(nroots, 0);
    int it_lp = 0;
    sigma_impl(c, ws, V, S, m, s, phase);
    k_dots(V, N, m, S, N, m, N, Gf, mmax, part, s);
    std::vector<double> thold(nroots, INFINITY), hrn(nroots * nroots + nroots), prev_rn(nroots, INFINITY);
    std::vector<char> mlp_on(nroots, (use_mlp && c->mlp_w) ? 1 : 0);
    std::vector<double> mlp_best(nroots, INFINITY);
    std::vector<int> mlp_stall(nroots, 0);
    if (use_mlp && c->mlp_w) mlp_weights_bf16(c->mlp_w, c->mlp_wb, s);
    std::vector<double> hY;
    int it = 0;
    for (;;) {
        ++it;
        // Rayleigh-Ritz on the (incrementally kept) Gram matrix
        k_copy2d(Gm, m, Gf, mmax, m, m, 1.0, 0.0, s);
        k_symmetrize(Gm, m, s);
        eig_small(Gm, m, ev, Y, s);
        k_sort_eig(ev, Y, m, 0, Gw, Gw + m, s);  // ascending, deterministic signs
        // Ritz vectors X = Y^T V, AX = Y^T S (first nroots columns of Y)
        k_copy2d(coef, nroots, Y, m, m, nroots, 1.0, 0.0, s);
        k_lincomb(Xr, N, nroots, V, N, m, coef, nroots, N, 1.0, 0.0, s);
        k_lincomb(AX, N, nroots, S, N, m, coef, nroots, N, 1.0, 0.0, s);
        k_copy(th, ev, nroots, s);
        k_residual(R, AX, Xr, th, nroots, N, s);
        k_dots(R, N, nroots, R, N, nroots, N, Gw, nroots, part, s);
        // the Ritz values travel with the residual Gram: one read-back per iteration
        k_copy(Gw + (long long)nroots * nroots, ev, nroots, s);
        d2h(hrn.data(), Gw, (size_t)(nroots * nroots + nroots) * sizeof(double), s);
        for (int k = 0; k < nroots; ++k) res.w[k] = hrn[(size_t)nroots * nroots + k];
        std::vector<int> todo;
        bool finite = true;
        for (int k = 0; k < nroots; ++k) {
            res.rn[k] = std::sqrt(std::max(0.0, hrn[k * nroots + k]));
            if (!std::isfinite(res.w[k]) || !std::isfinite(res.rn[k])) finite = false;
            bool ok = res.rn[k] <= conv && std::fabs(res.w[k] - thold[k]) <= conv;
            if (!ok) todo.push_back(k);
        }
        if (!finite) fail(-4, "davidson: non-finite Ritz value or residual");
        if (phase > 0) {
            // reduced-precision phase: stop at a tolerance set by the precision, or once every root still
            // above it has stalled (no 10% gain on its best residual in 4 iterations): slow progress of
            // some roots while others still improve is convergence, not the precision's noise floor
            ++it_lp;
            double scale = 1.0, rmax = 0.0;
            for (int k = 0; k < nroots; ++k) {
                scale = std::max(scale, std::fabs(res.w[k]));
                rmax = std::max(rmax, res.rn[k]);
            }
            const double tau = std::max(conv, (phase == 1 ? 1e-7 : 3e-4) * scale);
            bool all_stalled = true;
            for (int k = 0; k < nroots; ++k) {
                if (res.rn[k] < 0.9 * lp_best[k]) { lp_best[k] = res.rn[k]; lp_stall[k] = 0; } else ++lp_stall[k];
                if (res.rn[k] > tau && lp_stall[k] < 4) all_stalled = false;
            }
            if (rmax <= tau || all_stalled || it >= max_iter) {
                // residual correction in the next precision: restart from the Ritz vectors
                const int nkeep = std::min(m, nkeep_max);
                k_copy2d(coef, nkeep, Y, m, m, nkeep, 1.0, 0.0, s);
                k_lincomb(Vk, N, nkeep, V, N, m, coef, nkeep, N, 1.0, 0.0, s);
                k_copy(V, Vk, (long long)nkeep * N, s);
                m = nkeep;
                phase = (phase == 2 && c->Bvv32) ? 1 : 0;
                std::fill(lp_best.begin(), lp_best.end(), INFINITY);
                std::fill(lp_stall.begin(), lp_stall.end(), 0);
                if (phase == 0) {
                    res.iters_lowp = it_lp;
                    for (int k = 0; k < nroots; ++k) res.w_lowp.push_back(res.w[k]);
                }
                sigma_impl(c, ws, V, S, m, s, phase);
                k_dots(V, N, m, S, N, m, N, Gf, mmax, part, s);
                for (int k = 0; k < nroots; ++k) thold[k] = INFINITY;
                continue;
            }
        }
        if (verbosity() >= 2) {
            std::fprintf(stderr, "[adc3]   it %3d m %2d", it, m);
            for (int k = 0; k < nroots; ++k) std::fprintf(stderr, "  %.10f (%.1e)", res.w[k], res.rn[k]);
            std::fprintf(stderr, "\n");
        }
        res.iters = it;
        if (todo.empty() || it >= max_iter) {
            res.converged = todo.empty();
            break;
        }
        for (int k = 0; k < nroots; ++k) thold[k] = res.w[k];
        int nn = (int)todo.size();
        // collapse when the new block does not fit: keep the lowest nkeep Ritz vectors
        if (m + nn > mmax) {
            const int nkeep = std::min(m - 1, nkeep_max);
            k_copy2d(coef, nkeep, Y, m, m, nkeep, 1.0, 0.0, s);
            k_lincomb(Vk, N, nkeep, V, N, m, coef, nkeep, N, 1.0, 0.0, s);
            k_lincomb(Sk, N, nkeep, S, N, m, coef, nkeep, N, 1.0, 0.0, s);
            k_copy(V, Vk, (long long)nkeep * N, s);
            k_copy(S, Sk, (long long)nkeep * N, s);
            // the Gram of the Ritz basis is diag(theta)
            k_dots(V, N, nkeep, S, N, nkeep, N, Gf, mmax, part, s);
            m = nkeep;
        }
        nn = std::min(nn, mmax - m);
        if (nn <= 0) {
            res.converged = false;
            break;
        }
        // training data: features and Jacobi step at sampled elements, with the target the part of the
        // converged vector outside the current subspace, xf - V (V^T xf)
        if (rec) {
            for (int j = 0; j < nn && rec->G < rec->Gmax; ++j) {
                const int k = todo[j];
                const double rms = std::max(res.rn[k] / std::sqrt((double)N), 1e-300);
                const long long off = (long long)rec->G * rec->S;
                double* miss = Vk;  // free until the next collapse
                k_copy(miss, rec->xf + (long long)k * N, N, s);
                k_dots(V, N, m, miss, N, 1, N, Gw, 1, part, s);
                k_lincomb(miss, N, 1, V, N, m, Gw, 1, N, -1.0, 1.0, s);
                mlp_features_idx(R + (long long)k * N, c->diag, res.w[k], rms, c->eo, c->ev, c->o, c->v, rec->seed,
                                 rec->G, rec->S, N, miss, rec->F + off * 6, rec->A0 + off, rec->D + off, s);
                rec->G++;
            }
        }
        // preconditioned residuals of the unconverged roots -> V[m .. m+nn); learned steps for all
        // roots first, one flag word each, read back once
        double* Tn = V + (long long)m * N;
        bool any_mlp = false;
        for (int j = 0; j < nn; ++j) {
            const int k = todo[j];
            if (mlp_on[k]) {
                // Jacobi from here on if the learned steps made the residual grow, or stopped
                // reducing it (no 10% gain on its best value in 5 iterations)
                if (res.rn[k] < 0.9 * mlp_best[k]) {
                    mlp_best[k] = res.rn[k];
                    mlp_stall[k] = 0;
                } else {
                    ++mlp_stall[k];
                }
                if ((it > 1 && res.rn[k] > 2.0 * prev_rn[k]) || mlp_stall[k] >= 5) {
                    mlp_on[k] = 0;
                    VLOG("root %d: learned preconditioner disabled (residual %s)", k,
                         mlp_stall[k] >= 5 ? "stalled" : "grew");
                }
            }
            any_mlp = any_mlp || mlp_on[k];
        }
        if (any_mlp) k_fill((double*)mflag, (nn + 1) / 2, 0.0, s);
        // the exact 1p-block steps go out together, up to 16 vectors per launch
        Precond1p p1;
        p1.R = R; p1.T = Tn; p1.N = N; p1.Q = c->m11_Q; p1.w = c->m11_w; p1.th = th; p1.v = c->v;
        const bool p1_batch = c->v <= PRECOND_1P_VMAX;
        for (int j = 0; j < nn; ++j) {
            const int k = todo[j];
            if (mlp_on[k]) {
                const double rms = std::max(res.rn[k] / std::sqrt((double)N), 1e-300);
                mlp_precondition(R + (long long)k * N, c->diag, res.w[k], rms, c->eo, c->ev, c->o, c->v, N, c->mlp_w,
                                 c->mlp_wb, Tn + (long long)j * N, mflag + j, s);
            } else if (block1p) {
                // 1p block exactly: t1 = (M11 - theta)^-1 r1 through M11 = Q diag(w) Q^T; 2p1h diagonal
                const int v = c->v;
                if (p1_batch) {
                    p1.kidx[p1.nrow] = k;
                    p1.tidx[p1.nrow] = j;
                    if (++p1.nrow == 16) {
                        k_precond_1p(p1, s);
                        p1.nrow = 0;
                    }
                } else {
                    double* y = c->m11_tmp + (long long)v * v;
                    gemm_rm(1, v, v, 1.0, R + (long long)k * N, v, false, c->m11_Q, v, false, 0.0, y, v, s);
                    k_div_shift(y, c->m11_w, th + k, v, s);
                    gemm_rm(1, v, v, 1.0, y, v, false, c->m11_Q, v, true, 0.0, Tn + (long long)j * N, v, s);
                }
                k_precond(Tn + (long long)j * N + v, R + (long long)k * N + v, c->diag + v, th + k, 1, N - v, s);
            } else {
                k_precond(Tn + (long long)j * N, R + (long long)k * N, c->diag, th + k, 1, N, s);
                if (olsen) {
                    // Olsen: t = (D-theta)^-1 (r - eps x), eps = x.(D-theta)^-1 r / x.(D-theta)^-1 x
                    double* bx = Vk;  // free until the next collapse
                    k_precond(bx, Xr + (long long)k * N, c->diag, th + k, 1, N, s);
                    k_dots(Xr + (long long)k * N, N, 1, Tn + (long long)j * N, N, 1, N, small, 1, part, s);
                    k_dots(Xr + (long long)k * N, N, 1, bx, N, 1, N, small + 1, 1, part, s);
                    k_olsen(Tn + (long long)j * N, bx, small, N, s);
                }
            }
        }
        k_precond_1p(p1, s);
        if (any_mlp) {
            std::vector<unsigned int> hf(nn, 0);
            d2h(hf.data(), mflag, nn * sizeof(unsigned int), s);
            for (int j = 0; j < nn; ++j) {
                const int k = todo[j];
                if (mlp_on[k] && hf[j] != 0) {
                    mlp_on[k] = 0;
                    VLOG("root %d: learned preconditioner gave a non-finite step; Jacobi from here on", k);
                    k_precond(Tn + (long long)j * N, R + (long long)k * N, c->diag, th + k, 1, N, s);
                }
            }
        }
        for (int k = 0; k < nroots; ++k) prev_rn[k] = res.rn[k];
        const int acc = orthonormalise(Tn, nn, m, R);
        if (acc == 0) {
            res.converged = false;
            break;
        }
        sigma_impl(c, ws, V + (long long)m * N, S + (long long)m * N, acc, s, phase);
        {
            int at = g_nan_at.load();
            if (at > 0 && it >= at && g_nan_at.compare_exchange_strong(at, 0)) k_fill(S + (long long)m * N, N, NAN, s);
        }
        // new Gram columns V[0..m+acc) . S[m..m+acc), mirrored into the new rows
        k_dots(V, N, m + acc, S + (long long)m * N, N, acc, N, Gf + m, mmax, part, s);
        k_mirror_cols(Gf, mmax, m, acc, s);
        m += acc;
    }
    if (vec_out) k_copy(vec_out, Xr, (long long)nroots * N, s);
    HIPCHK(hipStreamSynchronize(s));
    ws.release(mark);
    return res;
}

// ---------------------------------------------------------------------------
// Lockstep block Davidson: many independent Davidson problems (instances of a ragged batch, or the
// per-root bases of one SS-FNO solve) advanced together, a fixed chunk of iterations per replay of one
// HIP graph that holds every active problem's iterations on its own stream.  The iteration has a fixed
// shape so that nothing in it needs the host: every iteration of a chunk adds the same nb directions (the
// preconditioned residuals of the roots not converged when the chunk began; those that converge within
// it, and directions lost to orthogonalisation, are zero vectors whose Gram rows are decoupled), the
// host knows the subspace size from the block widths, and the convergence flags, residual norms and
// Ritz values stay on the device until the chunk ends.
// ---------------------------------------------------------------------------
// iterations per graph replay (ADC3_DAV_CHUNK overrides; default 3)
static int lockstep_chunk() {
    static const int c = [] {
        const char* e = std::getenv("ADC3_DAV_CHUNK");
        const int v = (e && *e) ? std::atoi(e) : 3;
        return std::max(1, std::min(v, 64));
    }();
    return c;
}

struct LockJob {
    // problem (set by the caller)
    Ctx* c = nullptr;
    int nroots = 1, max_iter = 500, max_sub = 0;
    double conv = 1e-6;
    int pmode = 0;  // 0 Jacobi, 3 exact 1p block (ADC(2) contexts)
    int prec = 0;   // precision of the first phase (reduced-precision sigma until its floor, then FP64)
    const double* guess = nullptr;
    int nguess_in = 0;
    double* vec_out = nullptr;  // [nroots][N], nullable
    Arena* arena = nullptr;     // where the job's buffers are taken (jobs may share one)
    // state
    hipStream_t s = nullptr;
    long long N = 0;
    int mmax = 0, nb = 0, nguess = 0, nkeep = 0, m = 0, it = 0, phase = 0, it_lp = 0;
    double *V = nullptr, *S = nullptr, *Xr = nullptr, *AX = nullptr, *R = nullptr, *Gm = nullptr, *Gf = nullptr,
           *Gw = nullptr, *ev = nullptr, *Y = nullptr, *ev2 = nullptr, *Y2 = nullptr, *th = nullptr, *thold = nullptr,
           *coef = nullptr, *Vk = nullptr, *Sk = nullptr, *part = nullptr, *valid = nullptr, *active = nullptr,
           *status = nullptr, *tmp = nullptr, *Yb = nullptr, *gscr = nullptr, *nvalid = nullptr;
    // the block: nb <= nroots new directions per iteration, those of the roots idx[0..nb) (device), chosen at
    // each chunk boundary from the status; thg, actg their Ritz values and flags; Yr their raw 1p parts
    double *idx = nullptr, *thg = nullptr, *actg = nullptr, *Yr = nullptr;
    bool done = false;
    std::vector<double> lp_best;
    std::vector<int> lp_stall;
    DavResult res;
    long long sigma_builds = 0;
    size_t status_off = 0;  // offset (doubles) of this job's status in the host read-back buffer
    size_t idx_off = 0;     // offset (doubles) of this job's block indices in the pinned staging buffer
};

// does the problem's space hold the fixed block shape (guesses plus one block of nroots directions)?
static bool lock_fits(const LockJob& j) {
    const long long N = j.c->N;
    int mmax = j.max_sub > 0 ? j.max_sub : std::max(8 * j.nroots, 40);
    mmax = std::max(mmax, 2 * j.nroots + 1);
    mmax = (int)std::min<long long>(std::min(mmax, 96), N);
    return j.nroots <= 40 && mmax >= 2 * j.nroots;
}

static void lock_alloc(LockJob& j, Arena& ws) {
    Ctx* c = j.c;
    const long long N = c->N;
    j.N = N;
    if (j.nroots < 1 || j.nroots > N) fail(-1, "lockstep davidson: nroots out of range");
    if (j.nroots > 40) fail(-1, "lockstep davidson: at most 40 roots per problem");
    int mmax = j.max_sub > 0 ? j.max_sub : std::max(8 * j.nroots, 40);
    mmax = std::max(mmax, 2 * j.nroots + 1);
    j.mmax = (int)std::min<long long>(std::min(mmax, 96), N);
    j.nb = j.nroots;
    j.nguess = (int)std::min<long long>(N, std::min(j.nroots + 4, j.mmax - j.nb));
    j.nguess = std::max(j.nguess, j.nroots);
    if (j.nguess + j.nb > j.mmax) fail(-1, "lockstep davidson: space too small for the fixed block shape");
    j.nkeep = std::max(j.nroots, std::min(2 * j.nroots + 2, j.mmax - j.nb));
    const int mm = j.mmax, nr = j.nroots;
    j.V = take(ws, (long long)mm * N);
    j.S = take(ws, (long long)mm * N);
    j.Xr = take(ws, (long long)nr * N);
    j.AX = take(ws, (long long)nr * N);
    j.R = take(ws, (long long)nr * N);
    j.Vk = take(ws, (long long)j.nkeep * N);
    j.Sk = take(ws, (long long)j.nkeep * N);
    j.tmp = take(ws, (long long)std::max(j.nb, j.nguess) * N);
    j.Gm = take(ws, (long long)mm * mm);
    j.Gf = take(ws, (long long)mm * mm);
    j.Gw = take(ws, (long long)mm * mm + mm);
    j.ev = take(ws, mm);
    j.Y = take(ws, (long long)mm * mm);
    j.ev2 = take(ws, mm);
    j.Y2 = take(ws, (long long)mm * mm);
    j.th = take(ws, nr);
    j.thold = take(ws, nr);
    j.coef = take(ws, (long long)mm * mm);
    j.valid = take(ws, mm);
    j.active = take(ws, nr);
    j.status = take(ws, 2 + 3 * nr);
    j.idx = take(ws, nr);
    j.thg = take(ws, nr);
    j.actg = take(ws, nr);
    j.Yr = take(ws, (long long)nr * c->v);
    j.nvalid = take(ws, 1);
    j.Yb = take(ws, (long long)nr * c->v);
    j.part = take(ws, (long long)dots_partial_elems(mm, mm, N));
    j.gscr = take(ws, GEMM_SCRATCH);
    j.res.w.assign(nr, 0.0);
    j.res.rn.assign(nr, 0.0);
    j.lp_best.assign(nr, INFINITY);
    j.lp_stall.assign(nr, 0);
}

// GEMM scratch of a job while its work is issued (its own region: jobs run concurrently)
struct JobScratch {
    Arena a;
    GemmScratch g;
    explicit JobScratch(LockJob& j) : a(scratch_arena(j)), g(a, GEMM_SCRATCH) {}
    static Arena scratch_arena(LockJob& j) {
        Arena x;
        x.base = (char*)j.gscr;
        x.cap = GEMM_SCRATCH * sizeof(double) + 256;
        return x;
    }
};

// Tn[nn] against V[0..m) and within the block, two rounds of (classical Gram-Schmidt, Loewdin): directions
// whose Loewdin eigenvalue falls to <= 1e-14 become zero vectors and their valid flag 0 (valid[m..m+nn))
static void lock_ortho(LockJob& j, double* Tn, int nn, int m) {
    const long long N = j.N;
    hipStream_t s = j.s;
    k_dots(Tn, N, nn, Tn, N, nn, N, j.Gw, nn, j.part, s);
    k_rscale_rows(Tn, nn, N, j.Gw, nn, s);
    for (int round = 0; round < 2; ++round) {
        if (m > 0) {
            k_dots(j.V, N, m, Tn, N, nn, N, j.coef, nn, j.part, s);
            k_lincomb(Tn, N, nn, j.V, N, m, j.coef, nn, N, -1.0, 1.0, s);
        }
        k_dots(Tn, N, nn, Tn, N, nn, N, j.Gm, nn, j.part, s);
        k_symmetrize(j.Gm, nn, s);
        eig_small(j.Gm, nn, j.ev2, j.Y2, s);
        k_sort_eig(j.ev2, j.Y2, nn, 1, j.Gw, j.Gw + nn, s);
        k_lowdin_masked(j.coef, j.Y2, j.ev2, nn, 1e-14, j.valid + m, s);
        k_lincomb(j.tmp, N, nn, Tn, N, nn, j.coef, nn, N, 1.0, 0.0, s);
        k_copy(Tn, j.tmp, (long long)nn * N, s);
    }
}

static void lock_sigma(LockJob& j, const double* r, double* sg, int nvec) {
    Arena w = j.c->ws;
    const bool g = j.c->graphs;
    j.c->graphs = false;  // the pass is recorded into the lockstep graph, not captured on its own
    sigma_impl(j.c, w, r, sg, nvec, j.s, j.phase);
    j.c->graphs = g;
    j.sigma_builds += nvec;
}

// Rayleigh-Ritz over V[0..m) (masked directions decoupled), Ritz vectors, residuals, device status
static void lock_rr(LockJob& j) {
    const long long N = j.N;
    const int m = j.m, nr = j.nroots;
    hipStream_t s = j.s;
    k_copy2d(j.Gm, m, j.Gf, j.mmax, m, m, 1.0, 0.0, s);
    k_symmetrize(j.Gm, m, s);
    k_mask_gram(j.Gm, m, j.valid, j.nvalid, s);
    eig_small(j.Gm, m, j.ev, j.Y, s);
    k_sort_eig(j.ev, j.Y, m, 0, j.Gw, j.Gw + m, s);
    k_copy2d(j.coef, nr, j.Y, m, m, nr, 1.0, 0.0, s);
    k_lincomb(j.Xr, N, nr, j.V, N, m, j.coef, nr, N, 1.0, 0.0, s);
    k_lincomb(j.AX, N, nr, j.S, N, m, j.coef, nr, N, 1.0, 0.0, s);
    k_copy(j.th, j.ev, nr, s);
    k_residual(j.R, j.AX, j.Xr, j.th, nr, N, s);
    k_dots(j.R, N, nr, j.R, N, nr, N, j.Gw, nr, j.part, s);
    k_dav_status(j.Gw, nr, j.th, j.thold, j.conv, j.active, j.status, s);
    ++j.it;
}

// keep the nk lowest Ritz vectors of the last Rayleigh-Ritz (V, S and the Gram follow)
static void lock_collapse(LockJob& j, int nk, bool keep_sigma) {
    const long long N = j.N;
    hipStream_t s = j.s;
    k_copy2d(j.coef, nk, j.Y, j.m, j.m, nk, 1.0, 0.0, s);
    k_lincomb(j.Vk, N, nk, j.V, N, j.m, j.coef, nk, N, 1.0, 0.0, s);
    k_copy(j.V, j.Vk, (long long)nk * N, s);
    if (keep_sigma) {
        k_lincomb(j.Sk, N, nk, j.S, N, j.m, j.coef, nk, N, 1.0, 0.0, s);
        k_copy(j.S, j.Sk, (long long)nk * N, s);
        k_dots(j.V, N, nk, j.S, N, nk, N, j.Gf, j.mmax, j.part, s);
    }
    k_valid_first(j.valid, nk, j.nvalid, s);
    j.m = nk;
}

// one iteration, device work only: collapse when the block does not fit, expand by nb preconditioned
// residuals (zero for converged roots), sigma, Gram columns, Rayleigh-Ritz and status
static void lock_iterate(LockJob& j) {
    JobScratch scr(j);
    const long long N = j.N;
    hipStream_t s = j.s;
    Ctx* c = j.c;
    if (j.m + j.nb > j.mmax) lock_collapse(j, j.nkeep, true);
    double* Tn = j.V + (long long)j.m * N;
    // the block's roots: Ritz values, flags (and raw 1p residuals for the exact 1p step) gathered
    k_block_gather(j.thg, j.actg, j.pmode == 3 ? j.Yr : nullptr, c->v, j.th, j.active, j.R, N, j.idx, j.nb, s);
    k_precond_idx(Tn, j.R, c->diag, j.th, j.idx, j.nb, N, s);
    if (j.pmode == 3) {
        // 1p block exactly: t1 = Q (w - theta)^-1 Q^T r1 per root
        const int v = c->v;
        gemm_rm(j.nb, v, v, 1.0, j.Yr, v, false, c->m11_Q, v, false, 0.0, j.Yb, v, s);
        for (int k = 0; k < j.nb; ++k) k_div_shift(j.Yb + (long long)k * v, c->m11_w, j.thg + k, v, s);
        gemm_rm(j.nb, v, v, 1.0, j.Yb, v, false, c->m11_Q, v, true, 0.0, Tn, N, s);
    }
    k_rows_mask(Tn, j.nb, N, j.actg, s);
    lock_ortho(j, Tn, j.nb, j.m);
    lock_sigma(j, Tn, j.S + (long long)j.m * N, j.nb);
    {
        // failure-injection hook (eager iterations only, never recorded into a graph)
        int at = g_nan_at.load();
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (at > 0 && j.it + 1 >= at && hipStreamIsCapturing(s, &cap) == hipSuccess &&
            cap == hipStreamCaptureStatusNone && g_nan_at.compare_exchange_strong(at, 0))
            k_fill(j.S + (long long)j.m * N, N, NAN, s);
    }
    k_dots(j.V, N, j.m + j.nb, j.S + (long long)j.m * N, N, j.nb, N, j.Gf + j.m, j.mmax, j.part, s);
    k_mirror_cols(j.Gf, j.mmax, j.m, j.nb, s);
    j.m += j.nb;
    lock_rr(j);
}

// host-side state of one iteration without issuing it (a replay of a captured chunk)
static void lock_iterate_host(LockJob& j) {
    if (j.m + j.nb > j.mmax) j.m = j.nkeep;
    j.m += j.nb;
    j.sigma_builds += j.nb;
    ++j.it;
}

// eager start: guesses, first sigma block, Rayleigh-Ritz (the first iteration)
static void lock_start(LockJob& j) {
    JobScratch scr(j);
    Ctx* c = j.c;
    const long long N = j.N;
    hipStream_t s = j.s;
    j.phase = std::min(j.prec, c->prec);
    const int ng = j.guess ? std::min(j.nguess_in, j.nguess) : 0;
    std::vector<double> hd(N);
    d2h(hd.data(), c->diag, N * sizeof(double), s);
    const int kneed = j.nguess - ng;
    std::vector<std::pair<double, long long>> heap;
    heap.reserve(kneed + 1);
    for (long long i = 0; i < N && kneed > 0; ++i) {
        const std::pair<double, long long> e(hd[i], i);
        if ((int)heap.size() < kneed) {
            heap.push_back(e);
            std::push_heap(heap.begin(), heap.end());
        } else if (e < heap.front()) {
            std::pop_heap(heap.begin(), heap.end());
            heap.back() = e;
            std::push_heap(heap.begin(), heap.end());
        }
    }
    std::sort_heap(heap.begin(), heap.end());
    k_fill(j.V, (long long)j.nguess * N, 0.0, s);
    if (ng > 0) k_copy(j.V, j.guess, (long long)ng * N, s);
    std::vector<double> one(1, 1.0);
    for (int k = 0; k < kneed; ++k) h2d(j.V + (long long)(ng + k) * N + heap[k].second, one.data(), sizeof(double), s);
    if (j.pmode == 3 && !c->m11_eig) {
        const long long vv = (long long)c->v * c->v;
        k_copy(c->m11_tmp, c->M11, vv, s);
        eig_large(c->m11_tmp, c->v, c->m11_w, c->m11_Q, c->m11_tmp + vv + c->v, s);
        c->m11_eig = true;
    }
    lock_ortho(j, j.V, j.nguess, 0);
    j.m = j.nguess;
    lock_sigma(j, j.V, j.S, j.m);
    k_dots(j.V, N, j.m, j.S, N, j.m, N, j.Gf, j.mmax, j.part, s);
    k_fill(j.thold, j.nroots, INFINITY, s);
    lock_rr(j);
}

// restart from the Ritz vectors in the next precision (reduced-precision phase at its noise floor)
static void lock_restart(LockJob& j, int phase) {
    JobScratch scr(j);
    const long long N = j.N;
    lock_collapse(j, std::min(j.m, j.nkeep), false);
    j.phase = phase;
    lock_sigma(j, j.V, j.S, j.m);
    k_dots(j.V, N, j.m, j.S, N, j.m, N, j.Gf, j.mmax, j.part, j.s);
    k_fill(j.thold, j.nroots, INFINITY, j.s);
    lock_rr(j);
}

// Runs every job to convergence (or its max_iter).  Jobs start eagerly on streams of their own, then
// advance `chunk` iterations per replay of a graph of their own, launched on their own stream (so that
// the jobs run concurrently); after the replays every job's status comes back and the host decides
// restarts and the next blocks.  Graphs are kept per (job, subspace size, phase, chunk, block width),
// so a repeating collapse cycle replays them.
static void lockstep_run(std::vector<LockJob*>& jobs_in, hipStream_t caller, int chunk) {
    // spaces too small for the fixed shape (a few truncated virtuals) take the one-at-a-time Davidson
    std::vector<LockJob*> jobs;
    for (auto* j : jobs_in) {
        if (lock_fits(*j)) {
            jobs.push_back(j);
            continue;
        }
        const long long before = j->c->sigma_count;
        j->res = davidson_impl(j->c, *j->arena, j->nroots, j->conv, j->max_iter, j->max_sub, j->vec_out, caller,
                               j->prec, false, nullptr, j->guess, j->nguess_in, j->pmode);
        j->sigma_builds = j->c->sigma_count - before;
        j->done = true;
    }
    if (jobs.empty()) return;
    if (g_dry) {
        for (auto* j : jobs) {
            lock_alloc(*j, *j->arena);
            Arena w = j->c->ws;
            sigma_impl(j->c, w, dry_vec(), dry_vec(), std::min(NVMAX, j->nguess), nullptr, j->prec);
        }
        return;
    }
    const int nj = (int)jobs.size();
    size_t tot = 0;
    for (auto* j : jobs) {
        lock_alloc(*j, *j->arena);
        j->status_off = tot;
        tot += 2 + 3 * j->nroots;
        j->idx_off = tot;
        tot += j->nroots;
    }
    struct Res {
        hipStream_t main = nullptr;  // forks from the caller's stream into the jobs' streams and joins them back
        std::vector<hipStream_t> st;
        std::vector<hipEvent_t> ev;
        hipEvent_t fork = nullptr;
        double* host = nullptr;
        std::vector<std::map<std::string, hipGraphExec_t>> graphs;  // per job
        std::vector<std::set<std::string>> seen;  // per job: chunk shapes issued once without a graph
        ~Res() {
            for (auto& m : graphs)
                for (auto& kv : m) (void)hipGraphExecDestroy(kv.second);
            for (auto e : ev) (void)hipEventDestroy(e);
            if (fork) (void)hipEventDestroy(fork);
            for (auto x : st) (void)hipStreamDestroy(x);
            if (main) (void)hipStreamDestroy(main);
            if (host) (void)hipHostFree(host);
        }
    } rs;
    rs.graphs.resize(nj);
    rs.seen.resize(nj);
    HIPCHK(hipHostMalloc((void**)&rs.host, std::max<size_t>(tot, 1) * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&rs.fork, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&rs.main, hipStreamNonBlocking));
    hipStream_t main = rs.main;
    HIPCHK(hipEventRecord(rs.fork, caller));
    HIPCHK(hipStreamWaitEvent(main, rs.fork, 0));
    for (int i = 0; i < nj; ++i) {
        hipStream_t x = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        rs.st.push_back(x);
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        rs.ev.push_back(e);
        jobs[i]->s = x;
        HIPCHK(hipStreamWaitEvent(x, rs.fork, 0));
    }
    for (auto* j : jobs) lock_start(*j);
    auto read_status = [&](const std::vector<int>& ids, hipStream_t s) {
        for (int i : ids)
            HIPCHK(hipMemcpyAsync(rs.host + jobs[i]->status_off, jobs[i]->status,
                                  (2 + 3 * jobs[i]->nroots) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    };
    // the start's status: each job's own stream
    for (int i = 0; i < nj; ++i) read_status({i}, jobs[i]->s);
    // evaluation with restarts handled per job index
    auto step_eval = [&](int i) {
        LockJob& j = *jobs[i];
        for (;;) {
            const double* h = rs.host + j.status_off;
            const int nr = j.nroots;
            for (int k = 0; k < nr; ++k) {
                j.res.rn[k] = h[2 + k];
                j.res.w[k] = h[2 + nr + k];
            }
            if (h[1] == 0.0) fail(ADC3_ENUMERIC, "davidson: non-finite Ritz value or residual");
            if (j.phase > 0) {
                double scale = 1.0, rmax = 0.0;
                for (int k = 0; k < nr; ++k) {
                    scale = std::max(scale, std::fabs(j.res.w[k]));
                    rmax = std::max(rmax, j.res.rn[k]);
                }
                const double tau = std::max(j.conv, (j.phase == 1 ? 1e-7 : 3e-4) * scale);
                bool all_stalled = true;
                for (int k = 0; k < nr; ++k) {
                    if (j.res.rn[k] < 0.9 * j.lp_best[k]) { j.lp_best[k] = j.res.rn[k]; j.lp_stall[k] = 0; }
                    else j.lp_stall[k] += std::max(1, chunk);
                    if (j.res.rn[k] > tau && j.lp_stall[k] < 4) all_stalled = false;
                }
                if (rmax <= tau || all_stalled || j.it >= j.max_iter) {
                    const int next = (j.phase == 2 && j.c->Bvv32) ? 1 : 0;
                    if (next == 0) {
                        j.res.iters_lowp = j.it;
                        j.res.w_lowp = j.res.w;
                    }
                    std::fill(j.lp_best.begin(), j.lp_best.end(), INFINITY);
                    std::fill(j.lp_stall.begin(), j.lp_stall.end(), 0);
                    lock_restart(j, next);
                    read_status({i}, j.s);
                    continue;  // evaluate the restart's Rayleigh-Ritz
                }
                return;
            }
            if (h[0] != 0.0 || j.it >= j.max_iter) {
                j.done = true;
                j.res.converged = h[0] != 0.0;
                j.res.iters = j.it;
            }
            return;
        }
    };
    // the next chunk's block: the roots the status marks active, in root order (all of them when none is,
    // which only a phase that is about to restart can see); the indices go up on the job's stream
    auto set_block = [&](int i) {
        LockJob& j = *jobs[i];
        if (j.done) return;
        const double* h = rs.host + j.status_off;
        double* st = rs.host + j.idx_off;
        const int nr = j.nroots;
        int nb = 0;
        for (int k = 0; k < nr; ++k)
            if (h[2 + 2 * nr + k] != 0.0) st[nb++] = (double)k;
        if (nb == 0) {
            for (int k = 0; k < nr; ++k) st[k] = (double)k;
            nb = nr;
        }
        j.nb = nb;
        HIPCHK(hipMemcpyAsync(j.idx, st, nb * sizeof(double), hipMemcpyHostToDevice, j.s));
    };
    for (int i = 0; i < nj; ++i) {
        step_eval(i);
        set_block(i);
    }
    std::vector<std::set<int>> tuned(nj);  // (phase, block width) pairs a job has run eagerly
    // one graph per job and chunk shape, captured on and replayed on the job's own stream, so that the
    // jobs' chunks run concurrently (the nodes of one graph run one after another).  A job's first chunk
    // at a (precision, block width) runs eagerly, so that the ladder tuner settles its shapes before any
    // capture; a shape is captured the second time it comes up (a collapse cycle repeats its shapes), and
    // the first time its chunk is issued directly: a capture that is never replayed only costs host
    // time.  Each job is issued, waited for and evaluated by a host thread of its own, chunk after chunk
    // until it ends, without waiting for the other jobs' chunks (problems of different sizes and root
    // counts take chunks of different lengths).
    auto advance = [&](int i) {
        LockJob& j = *jobs[i];
        const int K = std::max(1, std::min(chunk, j.max_iter - j.it));
        if (tuned[i].insert(j.phase * 64 + j.nb).second) {
            for (int k = 0; k < K; ++k) lock_iterate(j);
        } else {
            const std::string key = std::to_string(j.m) + ":" + std::to_string(j.phase) + ":" +
                                    std::to_string(K) + ":" + std::to_string(j.nb);
            auto& graphs = rs.graphs[i];
            auto g = graphs.find(key);
            if (g == graphs.end() && rs.seen[i].insert(key).second) {
                for (int k = 0; k < K; ++k) lock_iterate(j);
            } else {
                if (g == graphs.end()) {
                    hipGraph_t gr = nullptr;
                    HIPCHK(hipStreamBeginCapture(j.s, hipStreamCaptureModeThreadLocal));
                    try {
                        for (int k = 0; k < K; ++k) lock_iterate(j);
                    } catch (...) {
                        // close the capture so that no stream is left capturing
                        hipGraph_t bad = nullptr;
                        (void)hipStreamEndCapture(j.s, &bad);
                        if (bad) (void)hipGraphDestroy(bad);
                        throw;
                    }
                    HIPCHK(hipStreamEndCapture(j.s, &gr));
                    hipGraphExec_t ex = nullptr;
                    HIPCHK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
                    HIPCHK(hipGraphDestroy(gr));
                    g = graphs.emplace(key, ex).first;
                } else {
                    for (int k = 0; k < K; ++k) lock_iterate_host(j);
                }
                HIPCHK(hipGraphLaunch(g->second, j.s));
            }
        }
        // the job's status after its chunk
        HIPCHK(hipMemcpyAsync(rs.host + j.status_off, j.status, (2 + 3 * j.nroots) * sizeof(double),
                              hipMemcpyDeviceToHost, j.s));
        HIPCHK(hipStreamSynchronize(j.s));
        step_eval(i);
        set_block(i);
    };
    std::atomic<bool> stop{false};
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    auto run = [&](int i) {
        HIPCHK(hipSetDevice(dev));  // the caller's device in every thread
        while (!jobs[i]->done && !stop.load()) advance(i);
    };
    std::vector<int> act;
    for (int i = 0; i < nj; ++i)
        if (!jobs[i]->done) act.push_back(i);
    if (act.size() == 1) {
        run(act[0]);
    } else if (!act.empty()) {
        std::vector<std::exception_ptr> errs(act.size());
        std::vector<std::thread> th;
        th.reserve(act.size() - 1);
        for (size_t t = 1; t < act.size(); ++t)
            th.emplace_back([&, t] {
                try {
                    run(act[t]);
                } catch (...) {
                    errs[t] = std::current_exception();
                    stop.store(true);
                }
            });
        try {
            run(act[0]);
        } catch (...) {
            errs[0] = std::current_exception();
            stop.store(true);
        }
        for (auto& x : th) x.join();
        for (auto& e : errs)
            if (e) std::rethrow_exception(e);
    }
    for (int i = 0; i < nj; ++i) {
        LockJob& j = *jobs[i];
        if (j.vec_out) k_copy(j.vec_out, j.Xr, (long long)j.nroots * j.N, j.s);
        HIPCHK(hipEventRecord(rs.ev[i], j.s));
        HIPCHK(hipStreamWaitEvent(main, rs.ev[i], 0));
    }
    HIPCHK(hipStreamSynchronize(main));
    HIPCHK(hipEventRecord(rs.fork, main));
    HIPCHK(hipStreamWaitEvent(caller, rs.fork, 0));
    for (auto* j : jobs) j->s = nullptr;
}

// ---------------------------------------------------------------------------
// SS-FNO / NAF pipeline (Sec. "Computational Details", steps 2-4f)
// ---------------------------------------------------------------------------
struct Blocks {
    double *Boo, *Bov, *Bvv;
    int X, o, v;
};

// D^EA(k) (eq 17, zeroth-order ISR of the ADC(2) eigenvector), spin averaged:
// 1/2 [r1 r1^T + sum_ci (x_aci x_bci + y_aci y_bci + x_cai x_cbi)],  y = x - x^T
static void ea_density(Arena& ws, const Ctx* c, const double* vec, double* D, hipStream_t s) {
    const int o = c->o, v = c->v;
    const long long vv = (long long)v * v, ovv = o * vv;
    const size_t mark = ws.mark();
    double* x = take(ws, ovv);
    double* y = take(ws, ovv);
    k_z_to_x(vec + v, x, nullptr, o, v, s);
    k_comb_t(y, x, o, v, 1.0, -1.0, s);
    gemm_rm(v, v, 1, 0.5, vec, 1, false, vec, v, false, 0.0, D, v, s);
    TV tx(x, {o, v, v}), ty(y, {o, v, v});
    ein(ws, "iac,ibc->ab", 0.5, tx, tx, 1.0, D, s);
    ein(ws, "iac,ibc->ab", 0.5, ty, ty, 1.0, D, s);
    ein(ws, "ica,icb->ab", 0.5, tx, tx, 1.0, D, s);
    ws.release(mark);
}

// Spectral amplitudes x = Y^T f (eqs 7-8) of one vector in the context's basis, x[o + v] (occupied
// orbitals first), with f_Ap = <Psi~_A| c+_p |Psi0> through second order in the 1p rows and first order
// in the 2p1h rows:  x_b = y1_b - (D^MP2 y1)_b / 2 (virtual b);  x_j = -(u1 y1)_j - sum_iab
// [(S + sqrt3 A) z]_iab T^ab_ji (occupied j).  tmp holds o v^2 doubles.
static void spectral_amplitudes(const Ctx* c, const double* vec, double* x, double* tmp, hipStream_t s) {
    const int o = c->o, v = c->v;
    const long long ovv = (long long)o * v * v;
    gemm_rm(1, v, v, -0.5, vec, v, false, c->Dmp2, v, false, 0.0, x + o, v, s);
    k_axpby(x + o, vec, v, 1.0, 1.0, s);
    k_fill(tmp, ovv, 0.0, s);
    k_d_to_z_add(tmp, vec + v, o, v, s);
    gemm_rm(1, o, (int)ovv, -1.0, tmp, ovv, false, c->T, ovv, true, 0.0, x, o, s);
    gemm_rm(1, o, v, -1.0, vec, v, false, c->u1, v, true, 1.0, x, o, s);
}

// Natural orbitals of D^SS (eq 9), kept eta > thr (eqs 10-11; thr <= 0 keeps all), recanonicalised
// (eqs 12-13), U = V~ Z (eq 14), for every root at once (Dss [nr][v][v]), the eigenproblems of all roots
// solved as batches (one launch per Jacobi round for the whole batch; the recanonicalisation in groups of
// roots with the same kept count).  U_all[k] holds U of root k as [v][vk_k], e_all[k] its vk_k energies
// (row stride v), vks[k] the kept count.
static void natural_orbitals_all(Arena& ws, const double* Dss, const double* ev, int v, double thr, int nr,
                                 double* U_all, double* e_all, std::vector<int>& vks, hipStream_t s,
                                 int keep_n = 0) {
    const long long vv = (long long)v * v;
    const size_t mark = ws.mark();
    double* A = take(ws, nr * vv);
    double* w = take(ws, (long long)nr * v);
    double* V = take(ws, nr * vv);
    double* wt = take(ws, v);
    double* Vt = take(ws, vv);
    double* scr = take(ws, (long long)eig_batched_scratch(v, nr));
    k_copy(A, Dss, nr * vv, s);
    for (int k = 0; k < nr; ++k) k_symmetrize(A + k * vv, v, s);
    eig_batched(A, v, nr, w, V, scr, s);
    for (int k = 0; k < nr; ++k) k_sort_eig(w + (long long)k * v, V + k * vv, v, 1, wt, Vt, s);  // descending
    std::vector<double> hw((size_t)nr * v);
    d2h(hw.data(), w, (size_t)nr * v * sizeof(double), s);
    vks.assign(nr, 0);
    for (int k = 0; k < nr; ++k) {
        if (g_dry || (keep_n <= 0 && !(thr > 0))) vks[k] = v;
        else if (keep_n > 0) vks[k] = std::min(keep_n, v);  // a fixed share of the virtuals, largest occupations
        else
            for (int a = 0; a < v; ++a) vks[k] += hw[(size_t)k * v + a] > thr;
    }
    // F~_k = V~_k^T diag(e) V~_k (V~_k = first vk_k columns of V_k), batched over roots with equal vk
    double* EV = take(ws, nr * vv);
    double* EVs = take(ws, vv);
    double* F = take(ws, nr * vv);
    double* Z = take(ws, nr * vv);
    double* en = take(ws, (long long)nr * v);
    double* zt = take(ws, vv);
    double* scr2 = take(ws, (long long)eig_batched_scratch(v, nr));
    std::vector<char> done(nr, 0);
    for (int k0 = 0; k0 < nr; ++k0) {
        const int vk = vks[k0];
        if (done[k0] || vk < 1) continue;
        std::vector<int> grp;
        for (int k = k0; k < nr; ++k)
            if (!done[k] && vks[k] == vk) { grp.push_back(k); done[k] = 1; }
        const long long kk = (long long)vk * vk;
        for (size_t j = 0; j < grp.size(); ++j) {
            double* EVk = EV + grp[j] * vv;
            k_copy2d(EVk, vk, V + grp[j] * vv, v, v, vk, 1.0, 0.0, s);
            k_scale_rows(EVs, EVk, ev, v, vk, s);
            gemm_rm(vk, vk, v, 1.0, EVk, vk, true, EVs, vk, false, 0.0, F + j * kk, vk, s);
            k_symmetrize(F + j * kk, vk, s);
        }
        eig_batched(F, vk, (int)grp.size(), en, Z, scr2, s);
        for (size_t j = 0; j < grp.size(); ++j) {
            const int k = grp[j];
            k_sort_eig(en + j * vk, Z + j * kk, vk, 0, wt, zt, s);
            double* U = U_all + k * vv;
            gemm_rm(v, vk, vk, 1.0, EV + k * vv, vk, false, Z + j * kk, vk, false, 0.0, U, vk, s);
            k_colsign(U, vk, v, vk, s);
            k_copy(e_all + (long long)k * v, en + j * vk, vk, s);
        }
    }
    ws.release(mark);
}

// New factor blocks in the truncated virtual basis: Bov U, U^T Bvv U (eqs 14-16).
static void transform_blocks(const Blocks& in, const double* U, int vk, Blocks& out, Arena& ws, hipStream_t s) {
    const int X = in.X, o = in.o, v = in.v;
    out.X = X; out.o = o; out.v = vk;
    out.Boo = in.Boo;
    out.Bov = take(ws, (long long)X * o * vk);
    out.Bvv = take(ws, (long long)X * vk * vk);
    gemm_rm(X * o, vk, v, 1.0, in.Bov, v, false, U, vk, false, 0.0, out.Bov, vk, s);
    const size_t mark = ws.mark();
    double* tmp = take(ws, (long long)X * v * vk);
    gemm_rm(X * v, vk, v, 1.0, in.Bvv, v, false, U, vk, false, 0.0, tmp, vk, s);
    Gemm g;
    g.M = vk; g.N = vk; g.K = v;
    g.A = U; g.sAm = 1; g.sAk = vk;
    g.B = tmp; g.sBk = vk; g.sBn = 1; g.bB0 = (long long)v * vk;
    g.C = out.Bvv; g.sCm = vk; g.sCn = 1; g.bC0 = (long long)vk * vk;
    for (int q0 = 0; q0 < X; q0 += 65535) {
        Gemm h = g;
        h.nb0 = std::min(65535, X - q0);
        h.B = tmp + (long long)q0 * v * vk;
        h.C = out.Bvv + (long long)q0 * vk * vk;
        gemm(h, s);
    }
    ws.release(mark);
}

// Natural auxiliary functions (eqs 27-29): W = J_vv J_vv^T, keep w >= thr (thr <= 0 keeps all).
// W is invariant under orthogonal rotations of the virtual basis: W_PQ = tr(B^P Pi B^Q Pi) with Pi
// the projector onto the kept virtuals.  When nothing is truncated (Pi = 1) every root has the
// same W, so the first root's eigenvectors are kept in `cache` and reused.
struct NafCache {
    double* N = nullptr;  // X x X, sorted eigenvectors
    double* w = nullptr;  // X eigenvalues
    bool valid = false;
};

static int naf_blocks(const Blocks& in, double thr, Blocks& out, Arena& ws, hipStream_t s, NafCache* cache = nullptr) {
    const int X = in.X, o = in.o, v = in.v;
    const long long vv = (long long)v * v;
    double* W = take(ws, (long long)X * X);
    double* w = take(ws, X);
    double* N = take(ws, (long long)X * X);
    if (cache && cache->valid) {
        k_copy(N, cache->N, (long long)X * X, s);
        k_copy(w, cache->w, X, s);
    } else {
        const size_t mark = ws.mark();
        double* wt = take(ws, X);
        double* Nt = take(ws, (long long)X * X);
        double* scr = take(ws, (long long)eig_large_scratch(X));
        gemm_rm(X, X, (int)vv, 1.0, in.Bvv, vv, false, in.Bvv, vv, true, 0.0, W, X, s);
        k_symmetrize(W, X, s);
        eig_large(W, X, w, N, scr, s);
        k_sort_eig(w, N, X, 1, wt, Nt, s);
        ws.release(mark);
        if (cache) {
            k_copy(cache->N, N, (long long)X * X, s);
            k_copy(cache->w, w, X, s);
            cache->valid = !g_dry;
        }
    }
    std::vector<double> hw(std::max(X, 1));
    d2h(hw.data(), w, X * sizeof(double), s);
    int xk = 0;
    if (g_dry || !(thr > 0)) xk = X;
    else
        for (int q = 0; q < X; ++q) xk += hw[q] >= thr;
    out.X = xk; out.o = o; out.v = v;
    out.Boo = take(ws, (long long)xk * o * o);
    out.Bov = take(ws, (long long)xk * o * v);
    out.Bvv = take(ws, (long long)xk * vv);
    if (xk > 0) {
        gemm_rm(xk, o * o, X, 1.0, N, X, true, in.Boo, (long long)o * o, false, 0.0, out.Boo, (long long)o * o, s);
        gemm_rm(xk, o * v, X, 1.0, N, X, true, in.Bov, (long long)o * v, false, 0.0, out.Bov, (long long)o * v, s);
        gemm_rm(xk, (int)vv, X, 1.0, N, X, true, in.Bvv, vv, false, 0.0, out.Bvv, vv, s);
    }
    return xk;
}

// The ADC(2) 1p block M11 = diag(e) - sym(P), P_ab = sum_klc (2T - T~)_kl^ac (kb|lc), of a basis (the same
// steps as the context build), into M11 [v][v].
static void m11_adc2(Arena& ws, const double* eo, const double* ev, const Blocks& B, double* M11, hipStream_t s) {
    const int o = B.o, v = B.v, X = B.X;
    const long long oo = (long long)o * o, ov = (long long)o * v, vv = (long long)v * v;
    const size_t mark = ws.mark();
    GemmScratch gscr(ws, GEMM_SCRATCH);
    double* ovov = take(ws, ov * ov);
    ein(ws, "Qia,Qjb->iajb", 1.0, TV(B.Bov, {X, o, v}), TV(B.Bov, {X, o, v}), 0.0, ovov, s);
    double* T = take(ws, oo * vv);
    k_amp_t(ovov, eo, ev, o, v, T, s);
    double* Tt2 = take(ws, oo * vv);
    k_comb_t(Tt2, T, oo, v, 2.0, -1.0, s);
    double* P = take(ws, vv);
    ein(ws, "klac,kblc->ab", 1.0, TV(Tt2, {o, o, v, v}), TV(ovov, {o, v, o, v}), 0.0, P, s);
    k_fill(M11, vv, 0.0, s);
    add_sym(M11, P, v, -1.0, s);
    k_add_diag(M11, ev, v, s);
    ws.release(mark);
}

struct SolveOut {
    std::vector<adc3_root_report> rep;
    bool all_conv = true;
};

// Pole strengths and Dyson-orbital coefficients from the spectral amplitudes xd[nroots][o + v] (canonical
// MO basis): each vector's sign fixed so that its largest-magnitude entry is positive (first on ties),
// P_k = sum_p x_kp^2 into the reports, the fixed vectors to dyson_out (device, nullable).
static void finish_amplitudes(double* xd, int nroots, int n, std::vector<adc3_root_report>& rep, double* dyson_out,
                              hipStream_t s) {
    std::vector<double> h((size_t)nroots * n);
    d2h(h.data(), xd, h.size() * sizeof(double), s);
    for (int k = 0; k < nroots; ++k) {
        double* x = h.data() + (size_t)k * n;
        int imax = 0;
        double ps = 0.0;
        for (int p = 0; p < n; ++p) {
            ps += x[p] * x[p];
            if (std::fabs(x[p]) > std::fabs(x[imax])) imax = p;
        }
        if (x[imax] < 0)
            for (int p = 0; p < n; ++p) x[p] = -x[p];
        rep[k].pole_strength = ps;
    }
    if (dyson_out) h2d(dyson_out, h.data(), h.size() * sizeof(double), s);
}

// Truncation of the virtual space asked for by the options (SS-FNO or MP2-FNO, by threshold or by
// share of the virtuals) or of the auxiliary basis (NAF)?
static bool truncates(double fno, double naf, const adc3_opts& op) {
    return fno > 0 || naf > 0 || op.fno_keep_frac > 0;
}

static SolveOut solve_impl(Arena& ws, const double* eo, const double* ev, const Blocks& B0, int nroots, double fno,
                           double naf, double conv, const adc3_opts& op, hipStream_t s) {
    const int o = B0.o, v = B0.v, X = B0.X;
    SolveOut out;
    out.rep.assign(nroots, adc3_root_report{});
    const int level = op.level;
    const double smx = level >= 3 ? op.sm_x : 1.0;
    // Davidson step per level: ADC(2) solves take the exact 1p block unless Jacobi or Olsen is
    // asked for (their 2p1h block is diagonal, so only the 1p block is approximated by the
    // diagonal step); ADC(3) solves take Jacobi, Olsen, or the learned step
    const int pm2 = (op.precond == 0 || op.precond == 2) ? op.precond : 3;
    const int pm3 = op.precond == 2 ? 2 : 0;
    // one ladder form for every ADC(3) context of the solve, chosen from the canonical size (so the
    // workspace plan holds for any truncation)
    const bool df = op.ladder == 2 || (op.ladder == 0 && ladder_df_auto(v));
    const long long N0 = v + (long long)o * v * v, vv0 = (long long)v * v;
    const int ng = op.init_guess ? (int)std::min<long long>(op.n_guess, N0) : 0;
    if (!truncates(fno, naf, op)) {
        const size_t mark = ws.mark();
        Ctx* c = build_ctx(ws, eo, ev, B0.Boo, B0.Bov, B0.Bvv, o, v, X, level, s, op.precision, df, smx);
        c->mlp_w = op.mlp_weights;
        c->graphs = op.sigma_graphs != 0;
        double* vecs = op.vectors_out ? op.vectors_out : take(ws, (long long)nroots * N0);
        DavResult r;
        if (op.lockstep == 1 && op.precond != 1 && op.precond != 2) {
            // the lockstep engine with one problem: fixed-shape iterations replayed from graphs
            LockJob j;
            j.c = c;
            j.nroots = nroots; j.conv = conv; j.max_iter = op.max_iter; j.max_sub = op.max_subspace;
            j.pmode = level >= 3 ? pm3 : pm2; j.prec = op.precision;
            j.guess = op.init_guess; j.nguess_in = ng; j.vec_out = vecs;
            j.arena = &ws;
            std::vector<LockJob*> jp{&j};
            const size_t mj = ws.mark();
            lockstep_run(jp, s, lockstep_chunk());
            ws.release(mj);
            r = j.res;
            c->sigma_count = j.sigma_builds;
        } else {
            r = davidson_impl(c, ws, nroots, conv, op.max_iter, op.max_subspace, vecs, s, op.precision,
                              op.precond == 1 && level >= 3, nullptr, op.init_guess, ng, level >= 3 ? pm3 : pm2);
        }
        {
            const size_t mx = ws.mark();
            GemmScratch gscr(ws, GEMM_SCRATCH);  // the amplitudes' long-K products split K across the chip
            double* xd = take(ws, (long long)nroots * (o + v));
            double* tmp = take(ws, (long long)o * v * v);
            for (int k = 0; k < nroots; ++k)
                spectral_amplitudes(c, vecs + (long long)k * N0, xd + (long long)k * (o + v), tmp, s);
            if (!g_dry) finish_amplitudes(xd, nroots, o + v, out.rep, op.dyson_out, s);
            ws.release(mx);
        }
        for (int k = 0; k < nroots; ++k) {
            auto& R = out.rep[k];
            R.omega = R.omega_uncorr = r.w[k];
            R.omega_lowp = r.w_lowp.empty() ? r.w[k] : r.w_lowp[k];
            R.iters_lowp = r.iters_lowp;
            R.resnorm = r.rn[k];
            R.err_bound = r.rn[k];
            R.nvir_kept = v;
            R.naux_kept = X;
            R.iters = r.iters;
            R.sigma_builds = k == 0 ? (int)c->sigma_count : 0;  // the solve's sigma builds, counted once
            R.sigma_builds_final = R.sigma_builds;
        }
        out.all_conv = r.converged;
        delete c;
        ws.release(mark);
        return out;
    }
    // Natural-orbital bases: one per root from D^SS(k) = D^MP2 + D^EA(k) (state-specific, eq 17), or
    // one shared by all roots from D^MP2 alone (ground-state MP2-FNO)
    const bool shared = op.fno_mode == 1;
    const int nb = shared ? 1 : nroots;
    const int keep_n = op.fno_keep_frac > 0 ? (int)std::max(1.0, std::ceil(op.fno_keep_frac * v - 1e-9)) : 0;
    // steps 2-3: canonical MP2 density and canonical ADC(2) roots; the canonical context is released
    // once the densities of all bases (steps 4a-4b) are formed
    const size_t mark0 = ws.mark();
    double* Y2 = take(ws, (long long)nroots * N0);
    double* Dss = take(ws, (long long)nb * vv0);
    double* xd = take(ws, (long long)nroots * (o + v));  // spectral amplitudes, canonical MO basis
    DavResult r2;
    int sig0 = 0;
    {
        const size_t mc0 = ws.mark();
        Ctx* c0 = build_ctx(ws, eo, ev, B0.Boo, B0.Bov, B0.Bvv, o, v, X, 2, s, op.precision);
        c0->graphs = op.sigma_graphs != 0;
        r2 = davidson_impl(c0, ws, nroots, conv, op.max_iter, op.max_subspace, Y2, s, op.precision, false, nullptr,
                           op.init_guess, ng, pm2);
        if (op.vectors_out) k_copy(op.vectors_out, Y2, (long long)nroots * N0, s);
        GemmScratch gscr(ws, GEMM_SCRATCH);
        for (int b = 0; b < nb; ++b) {
            double* D = Dss + (long long)b * vv0;
            if (shared) {
                k_copy(D, c0->Dmp2, vv0, s);                               // MP2-FNO: D^MP2 only
            } else {
                ea_density(ws, c0, Y2 + (long long)b * N0, D, s);          // 4a
                k_axpby(D, c0->Dmp2, vv0, 1.0, 1.0, s);                     // 4b
            }
        }
        sig0 = (int)c0->sigma_count;
        delete c0;
        ws.release(mc0);
    }
    out.all_conv = out.all_conv && r2.converged;
    VLOG("canonical ADC(2): %d roots, %d iterations, lowest %.10f", nroots, r2.iters, r2.w[0]);
    // steps 4c-4d for every basis: natural orbitals, truncation and recanonicalisation
    double* U_all = take(ws, (long long)nb * vv0);
    double* e_all = take(ws, (long long)nb * v);
    std::vector<int> vks;
    natural_orbitals_all(ws, Dss, ev, v, fno, nb, U_all, e_all, vks, s, keep_n);
    NafCache naf_cache;
    if (naf > 0) {
        naf_cache.N = take(ws, (long long)X * X);
        naf_cache.w = take(ws, X);
    }
    // step 4 for all bases: one after the other (engine 0); or each basis's steps on a host thread and
    // stream of its own (engine 2: opts.lockstep 2, and the default -1 whenever there are two bases or more
    // and their stored ladders, at the untruncated size, take at most the stored ladder's budget of 96 GB
    // together); or all bases' truncated ADC(2) solves in one lockstep block Davidson, then all their ADC(3)
    // solves in another (engine 1: opts.lockstep 1; not with the learned and Olsen steps).  Planning and the
    // solve take the same decision.
    const bool df_all = op.ladder == 2 || (op.ladder == 0 && ladder_df_auto(v));
    const double lock_ladder_bytes = (double)nb * 4.0 * (double)v * v * v * v;
    const bool together_auto = nb >= 2 && !df_all && lock_ladder_bytes <= 96e9;
    const int engine = (op.lockstep == 1 && op.precond != 1 && op.precond != 2) ? 1
                       : (op.lockstep == 2 || (op.lockstep < 0 && together_auto)) ? 2
                                                                                   : 0;
    // the truncated ADC(2) solves precondition with the exact 1p block: with the bases one after another,
    // the eigendecompositions of the bases' M11 solved as batches (bases with equal kept counts together)
    // before the per-basis solves, where that pays and costs no second NAF eigensolver: kept count above the
    // one-workgroup solver's size and the NAF result shared (nothing truncated) or not asked for.  With each
    // basis on a thread of its own (engine 2), each context solves its own M11 on its stream, beside the
    // other bases' work, instead of in a batch (and a second pass over the blocks) before the threads start.
    double* m11Q = nullptr;
    double* m11w = nullptr;
    std::vector<char> m11_pre(nb, 0);
    for (int b = 0; b < nb; ++b)
        m11_pre[b] = engine != 2 && pm2 == 3 && vks[b] > 96 && (!(naf > 0) || vks[b] == v);
    if (std::count(m11_pre.begin(), m11_pre.end(), 1) >= 2) {
        m11Q = take(ws, (long long)nb * vv0);
        m11w = take(ws, (long long)nb * v);
        const size_t mm = ws.mark();
        double* A = take(ws, (long long)nb * vv0);
        double* w = take(ws, (long long)nb * v);
        double* Q = take(ws, (long long)nb * vv0);
        double* scr = take(ws, (long long)eig_batched_scratch(v, nb));
        std::vector<char> done(nb, 0);
        for (int b0 = 0; b0 < nb; ++b0) {
            const int vk = vks[b0];
            if (done[b0] || !m11_pre[b0]) continue;
            std::vector<int> grp;
            for (int b = b0; b < nb; ++b)
                if (!done[b] && m11_pre[b] && vks[b] == vk) { grp.push_back(b); done[b] = 1; }
            const long long kk = (long long)vk * vk;
            for (size_t j = 0; j < grp.size(); ++j) {
                const size_t mb = ws.mark();
                GemmScratch gscr(ws, GEMM_SCRATCH);
                Blocks Bt, Bn;
                transform_blocks(B0, U_all + (long long)grp[j] * vv0, vk, Bt, ws, s);
                Bn = Bt;
                if (naf > 0) naf_blocks(Bt, naf, Bn, ws, s, vk == v ? &naf_cache : nullptr);
                m11_adc2(ws, eo, e_all + (long long)grp[j] * v, Bn, A + j * kk, s);
                ws.release(mb);
            }
            eig_batched(A, vk, (int)grp.size(), w, Q, scr, s);
            for (size_t j = 0; j < grp.size(); ++j) {
                k_copy(m11Q + (long long)grp[j] * vv0, Q + j * kk, kk, s);
                k_copy(m11w + (long long)grp[j] * v, w + (long long)j * vk, vk, s);
            }
        }
        ws.release(mm);
    }
    auto run_jobs = [&](std::vector<LockJob*>& jp) {
        const size_t mj = ws.mark();
        lockstep_run(jp, s, lockstep_chunk());
        ws.release(mj);
    };
    if (engine == 1) {
        GemmScratch gscr(ws, GEMM_SCRATCH);
        std::vector<Blocks> Bn(nb);
        std::vector<int> xks(nb, X);
        std::vector<long long> Nks(nb);
        std::vector<double*> carried(nb), Y2k(nb);
        for (int b = 0; b < nb; ++b) {
            const int vk = vks[b];
            if (vk < 1) fail(ADC3_EINVAL, "SS-FNO threshold removes every virtual orbital");
            const double* U = U_all + (long long)b * vv0;
            Blocks Bt;
            transform_blocks(B0, U, vk, Bt, ws, s);
            Bn[b] = Bt;
            if (naf > 0) xks[b] = naf_blocks(Bt, naf, Bn[b], ws, s, vk == v ? &naf_cache : nullptr);
            const long long Nk = vk + (long long)o * vk * vk;
            if (nroots > Nk) fail(ADC3_EINVAL, "truncated space smaller than nroots");
            Nks[b] = Nk;
            carried[b] = take(ws, (long long)nroots * Nk);
            Y2k[b] = take(ws, (long long)nroots * Nk);
            const size_t mt = ws.mark();
            double* tmp = take(ws, (long long)o * v * vk);
            for (int q = 0; q < nroots; ++q) {
                const double* yq = Y2 + (long long)q * N0;
                double* cq = carried[b] + (long long)q * Nk;
                gemm_rm(1, vk, v, 1.0, yq, v, false, U, vk, false, 0.0, cq, vk, s);
                gemm_rm(o * v, vk, v, 1.0, yq + v, v, false, U, vk, false, 0.0, tmp, vk, s);
                Gemm g;
                g.M = vk; g.N = vk; g.K = v;
                g.A = U; g.sAm = 1; g.sAk = vk;
                g.B = tmp; g.sBk = vk; g.sBn = 1; g.bB0 = (long long)v * vk;
                g.C = cq + vk; g.sCm = vk; g.sCn = 1; g.bC0 = (long long)vk * vk;
                g.nb0 = o;
                gemm(g, s);
            }
            ws.release(mt);
        }
        std::vector<std::vector<int>> ks(nb);
        for (int b = 0; b < nb; ++b) {
            if (shared)
                for (int k = 0; k < nroots; ++k) ks[b].push_back(k);
            else
                ks[b].push_back(b);
        }
        std::vector<int> match(nroots, 0);
        std::vector<DavResult> a2(nb);
        std::vector<long long> sig(nb, 0), sig3(nb, 0);  // per basis: all its solves, its final-level solve
        {
            const size_t m2 = ws.mark();
            std::vector<Ctx*> c2(nb, nullptr);
            std::vector<LockJob> jobs(nb);
            std::vector<LockJob*> jp;
            for (int b = 0; b < nb; ++b) {
                c2[b] = build_ctx(ws, eo, e_all + (long long)b * v, Bn[b].Boo, Bn[b].Bov, Bn[b].Bvv, o, vks[b],
                                  Bn[b].X, 2, s, op.precision);
                c2[b]->graphs = op.sigma_graphs != 0;
                if (m11Q && m11_pre[b]) {
                    k_copy(c2[b]->m11_Q, m11Q + (long long)b * vv0, (long long)vks[b] * vks[b], s);
                    k_copy(c2[b]->m11_w, m11w + (long long)b * v, vks[b], s);
                    c2[b]->m11_eig = true;
                }
            }
            for (int b = 0; b < nb; ++b) {
                LockJob& j = jobs[b];
                j.c = c2[b];
                j.nroots = nroots; j.conv = conv; j.max_iter = op.max_iter; j.max_sub = op.max_subspace;
                j.pmode = pm2; j.prec = op.precision;
                j.guess = carried[b]; j.nguess_in = nroots; j.vec_out = Y2k[b];
                j.arena = &ws;
                jp.push_back(&j);
            }
            run_jobs(jp);
            for (int b = 0; b < nb; ++b) {
                a2[b] = jobs[b].res;
                sig[b] += jobs[b].sigma_builds;
                out.all_conv = out.all_conv && a2[b].converged;
            }
            // overlaps of the truncated ADC(2) vectors with the carried canonical ones
            for (int b = 0; b < nb; ++b) {
                const size_t mo = ws.mark();
                double* ovl = take(ws, (long long)nroots * nroots);
                double* part = take(ws, (long long)dots_partial_elems(nroots, nroots, Nks[b]));
                k_dots(carried[b], Nks[b], nroots, Y2k[b], Nks[b], nroots, Nks[b], ovl, nroots, part, s);
                std::vector<double> hov((size_t)nroots * nroots);
                d2h(hov.data(), ovl, hov.size() * sizeof(double), s);
                for (int k : ks[b]) {
                    match[k] = k;
                    if (!g_dry) {
                        int m = 0;
                        for (int q = 1; q < nroots; ++q)
                            if (std::fabs(hov[(size_t)k * nroots + q]) > std::fabs(hov[(size_t)k * nroots + m])) m = q;
                        match[k] = m;
                    }
                    out.rep[k].omega_adc2_fno = a2[b].w[match[k]];
                }
                ws.release(mo);
            }
            for (int b = 0; b < nb; ++b) delete c2[b];
            ws.release(m2);
        }
        {
            const size_t m3 = ws.mark();
            std::vector<Ctx*> c3(nb, nullptr);
            std::vector<double*> X3(nb);
            std::vector<int> nr3(nb, 1);
            for (int b = 0; b < nb; ++b) {
                c3[b] = build_ctx(ws, eo, e_all + (long long)b * v, Bn[b].Boo, Bn[b].Bov, Bn[b].Bvv, o, vks[b],
                                  Bn[b].X, level, s, op.precision, df, smx);
                c3[b]->mlp_w = op.mlp_weights;
                c3[b]->graphs = op.sigma_graphs != 0;
                int mm = 0;
                for (int k : ks[b]) mm = std::max(mm, match[k]);
                nr3[b] = g_dry ? nroots : std::min(nroots, mm + 1);
                X3[b] = take(ws, (long long)nr3[b] * Nks[b]);
            }
            std::vector<LockJob> jobs(nb);
            std::vector<LockJob*> jp;
            for (int b = 0; b < nb; ++b) {
                LockJob& j = jobs[b];
                j.c = c3[b];
                j.nroots = nr3[b]; j.conv = conv; j.max_iter = op.max_iter; j.max_sub = op.max_subspace;
                j.pmode = level >= 3 ? pm3 : pm2; j.prec = op.precision;
                j.guess = Y2k[b]; j.nguess_in = nroots; j.vec_out = X3[b];
                j.arena = &ws;
                jp.push_back(&j);
            }
            run_jobs(jp);
            const size_t mx = ws.mark();
            for (int b = 0; b < nb; ++b) {
                const DavResult& a3 = jobs[b].res;
                const int vk = vks[b];
                sig[b] += jobs[b].sigma_builds;
                sig3[b] += jobs[b].sigma_builds;
                out.all_conv = out.all_conv && a3.converged;
                double* xk = take(ws, o + vk);
                double* tmp = take(ws, (long long)o * vk * vk);
                const double* U = U_all + (long long)b * vv0;
                for (int k : ks[b]) {
                    auto& R = out.rep[k];
                    const int m = match[k];
                    R.omega_adc2_can = r2.w[k];
                    R.omega_uncorr = a3.w[m];
                    R.omega_lowp = a3.w_lowp.empty() ? a3.w[m] : a3.w_lowp[m];
                    R.iters_lowp = a3.iters_lowp;
                    R.resnorm = a3.rn[m];
                    R.iters = a3.iters;
                    R.nvir_kept = vk;
                    R.naux_kept = xks[b];
                    R.omega = R.omega_uncorr + (op.fno_correction ? (R.omega_adc2_can - R.omega_adc2_fno) : 0.0);
                    R.err_bound = a3.rn[m] + (op.fno_correction ? r2.rn[k] + a2[b].rn[m] : 0.0);
                    double* xo = xd + (long long)k * (o + v);
                    spectral_amplitudes(c3[b], X3[b] + (long long)m * Nks[b], xk, tmp, s);
                    k_copy(xo, xk, o, s);
                    gemm_rm(1, v, vk, 1.0, xk + o, vk, false, U, vk, true, 0.0, xo + o, v, s);
                }
                ws.release(mx);
            }
            for (int b = 0; b < nb; ++b) delete c3[b];
            ws.release(m3);
        }
        // counted per basis, on the first root it serves (as one basis at a time does)
        for (int b = 0; b < nb; ++b)
            for (size_t j = 0; j < ks[b].size(); ++j) {
                out.rep[ks[b][j]].sigma_builds = j == 0 ? (int)sig[b] : 0;
                out.rep[ks[b][j]].sigma_builds_final = j == 0 ? (int)sig3[b] : 0;
            }
    }
    // step 4 for one basis once its blocks are formed: the roots it serves (root b for a state-specific
    // basis, all for a shared one), its truncated ADC(2) and ADC(3) solves and eq 30, its buffers taken from
    // `ar` and its work issued on `st`.  Returns whether both solves converged.
    auto run_basis = [&](int b, const Blocks& Bn, int xk, Arena& ar, hipStream_t st) -> bool {
        bool conv_b = true;
        GemmScratch gscr(ar, GEMM_SCRATCH);
        std::vector<int> ks;
        if (shared)
            for (int k = 0; k < nroots; ++k) ks.push_back(k);
        else
            ks.push_back(b);
        const double* U = U_all + (long long)b * vv0;
        const double* enew = e_all + (long long)b * v;
        const int vk = vks[b];
        const long long Nk = vk + (long long)o * vk * vk;
        if (nroots > Nk) fail(ADC3_EINVAL, "truncated space smaller than nroots");
        int sig = 0, sig3 = 0;
        std::vector<int> match(nroots, 0);
        // the canonical ADC(2) vectors carried into the truncated basis (r1 U, U^T z_i U): vector k is
        // the reference for root matching, all of them start the truncated ADC(2) solve, whose vectors
        // in turn start the truncated ADC(3) solve
        double* carried = take(ar, (long long)nroots * Nk);
        double* Y2k = take(ar, (long long)nroots * Nk);
        {
            const size_t mt = ar.mark();
            double* tmp = take(ar, (long long)o * v * vk);
            for (int q = 0; q < nroots; ++q) {
                const double* yq = Y2 + (long long)q * N0;
                double* cq = carried + (long long)q * Nk;
                gemm_rm(1, vk, v, 1.0, yq, v, false, U, vk, false, 0.0, cq, vk, st);
                gemm_rm(o * v, vk, v, 1.0, yq + v, v, false, U, vk, false, 0.0, tmp, vk, st);
                Gemm g;
                g.M = vk; g.N = vk; g.K = v;
                g.A = U; g.sAm = 1; g.sAk = vk;
                g.B = tmp; g.sBk = vk; g.sBn = 1; g.bB0 = (long long)v * vk;
                g.C = cq + vk; g.sCm = vk; g.sCn = 1; g.bC0 = (long long)vk * vk;
                g.nb0 = o;
                gemm(g, st);
            }
            ar.release(mt);
        }
        DavResult a2;
        {
            double* ovl = take(ar, (long long)nroots * nroots);
            double* part = take(ar, (long long)dots_partial_elems(nroots, nroots, Nk));
            const size_t m2 = ar.mark();
            Ctx* c2 = build_ctx(ar, eo, enew, Bn.Boo, Bn.Bov, Bn.Bvv, o, vk, Bn.X, 2, st, op.precision);
            c2->graphs = op.sigma_graphs != 0;
            if (m11Q && m11_pre[b]) {
                k_copy(c2->m11_Q, m11Q + (long long)b * vv0, (long long)vk * vk, st);
                k_copy(c2->m11_w, m11w + (long long)b * v, vk, st);
                c2->m11_eig = true;
            }
            a2 = davidson_impl(c2, ar, nroots, conv, op.max_iter, op.max_subspace, Y2k, st, op.precision, false,
                               nullptr, carried, nroots, pm2);
            // overlaps of the truncated ADC(2) vectors with every carried canonical vector: ovl[k][q]
            k_dots(carried, Nk, nroots, Y2k, Nk, nroots, Nk, ovl, nroots, part, st);
            std::vector<double> hov((size_t)nroots * nroots);
            d2h(hov.data(), ovl, hov.size() * sizeof(double), st);
            for (int k : ks) {
                match[k] = k;
                if (!g_dry) {
                    int m = 0;
                    for (int q = 1; q < nroots; ++q)
                        if (std::fabs(hov[(size_t)k * nroots + q]) > std::fabs(hov[(size_t)k * nroots + m])) m = q;
                    match[k] = m;
                }
                out.rep[k].omega_adc2_fno = a2.w[match[k]];
                VLOG("root %d: truncated ADC(2) %d iterations, matched root %d (overlap %.4f)", k, a2.iters,
                     match[k], std::fabs(hov[(size_t)k * nroots + match[k]]));
            }
            conv_b = conv_b && a2.converged;
            sig += (int)c2->sigma_count;
            delete c2;
            ar.release(m2);
        }
        {
            const size_t m3 = ar.mark();
            Ctx* c3 = build_ctx(ar, eo, enew, Bn.Boo, Bn.Bov, Bn.Bvv, o, vk, Bn.X, level, st, op.precision, df, smx);
            c3->mlp_w = op.mlp_weights;
            c3->graphs = op.sigma_graphs != 0;
            // only the roots up to the highest matched one of this basis are needed
            int mmax = 0;
            for (int k : ks) mmax = std::max(mmax, match[k]);
            const int nr3 = std::min(nroots, mmax + 1);
            double* X3 = take(ar, (long long)nr3 * Nk);
            DavResult a3 = davidson_impl(c3, ar, nr3, conv, op.max_iter, op.max_subspace, X3, st, op.precision,
                                         op.precond == 1, nullptr, Y2k, nroots, level >= 3 ? pm3 : pm2);
            {
                // spectral amplitudes of the matched roots in this basis, virtual part carried back to the
                // canonical virtuals through U (x_p = sum_a U[p][a] x~_a)
                const size_t mx = ar.mark();
                double* xk = take(ar, o + vk);
                double* tmp = take(ar, (long long)o * vk * vk);
                for (int k : ks) {
                    double* xo = xd + (long long)k * (o + v);
                    spectral_amplitudes(c3, X3 + (long long)match[k] * Nk, xk, tmp, st);
                    k_copy(xo, xk, o, st);
                    gemm_rm(1, v, vk, 1.0, xk + o, vk, false, U, vk, true, 0.0, xo + o, v, st);
                }
                ar.release(mx);
            }
            for (int k : ks) {
                auto& R = out.rep[k];
                const int m = match[k];
                R.omega_adc2_can = r2.w[k];
                R.omega_uncorr = a3.w[m];
                R.omega_lowp = a3.w_lowp.empty() ? a3.w[m] : a3.w_lowp[m];
                R.iters_lowp = a3.iters_lowp;
                VLOG("root %d: truncated ADC(3) %d iterations, omega %.10f, |r| %.2e", k, a3.iters, a3.w[m], a3.rn[m]);
                R.resnorm = a3.rn[m];
                R.iters = a3.iters;
                R.nvir_kept = vk;
                R.naux_kept = xk;
                R.omega = R.omega_uncorr + (op.fno_correction ? (R.omega_adc2_can - R.omega_adc2_fno) : 0.0);  // eq 30
                // each of the three eigenvalues lies within its residual norm of an eigenvalue of its matrix
                R.err_bound = a3.rn[m] + (op.fno_correction ? r2.rn[k] + a2.rn[m] : 0.0);
            }
            conv_b = conv_b && a3.converged;
            sig += (int)c3->sigma_count;
            sig3 = (int)c3->sigma_count;
            delete c3;
            ar.release(m3);
        }
        for (size_t j = 0; j < ks.size(); ++j) {
            out.rep[ks[j]].sigma_builds = j == 0 ? sig : 0;
            out.rep[ks[j]].sigma_builds_final = j == 0 ? sig3 : 0;
        }
        return conv_b;
    };
    // 4c-4e for basis b: its blocks in the kept natural orbitals, then the NAF truncation (the NAF
    // eigensolver's result is shared by the bases that keep every virtual)
    auto prep_basis = [&](int b, Blocks& Bn) -> int {
        const int vk = vks[b];
        if (vk < 1) fail(ADC3_EINVAL, "SS-FNO threshold removes every virtual orbital");
        GemmScratch gscr(ws, GEMM_SCRATCH);
        Blocks Bt;
        transform_blocks(B0, U_all + (long long)b * vv0, vk, Bt, ws, s);
        Bn = Bt;
        int xk = X;
        if (naf > 0) xk = naf_blocks(Bt, naf, Bn, ws, s, vk == v ? &naf_cache : nullptr);
        VLOG("basis %d: kept %d virtuals, %d auxiliary functions", b, vk, xk);
        return xk;
    };
    if (engine == 0) {
        for (int b = 0; b < nb; ++b) {
            const size_t mark = ws.mark();
            Blocks Bn;
            const int xk = prep_basis(b, Bn);
            const bool cb = run_basis(b, Bn, xk, ws, s);
            out.all_conv = out.all_conv && cb;
            ws.release(mark);
        }
    } else if (engine == 2) {
        // every basis's blocks first, on the caller's stream; then each basis's solves on a host thread and a
        // stream of its own, in a slice of the workspace sized by a dry run of the same steps, so that one
        // basis's context setup overlaps the other bases' Davidsons
        std::vector<Blocks> Bn(nb);
        std::vector<int> xks(nb, X);
        for (int b = 0; b < nb; ++b) xks[b] = prep_basis(b, Bn[b]);
        std::vector<Arena> sub(nb);
        for (int b = 0; b < nb; ++b) {
            const bool was = g_dry;
            g_dry = true;
            Arena count;
            run_basis(b, Bn[b], xks[b], count, nullptr);
            g_dry = was;
            const size_t bytes = (count.peak + 4096 + 255) / 256 * 256;
            sub[b].base = ws.take<char>(bytes);
            sub[b].cap = bytes;
        }
        if (!g_dry) {
            struct Res {
                std::vector<hipStream_t> st;
                std::vector<hipEvent_t> ev;
                hipEvent_t fork = nullptr;
                ~Res() {
                    for (auto e : ev) (void)hipEventDestroy(e);
                    if (fork) (void)hipEventDestroy(fork);
                    for (auto x : st) (void)hipStreamDestroy(x);
                }
            } rs;
            int dev = 0;
            HIPCHK(hipGetDevice(&dev));
            HIPCHK(hipEventCreateWithFlags(&rs.fork, hipEventDisableTiming));
            HIPCHK(hipEventRecord(rs.fork, s));
            for (int b = 0; b < nb; ++b) {
                hipStream_t x = nullptr;
                HIPCHK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
                rs.st.push_back(x);
                hipEvent_t e = nullptr;
                HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                rs.ev.push_back(e);
                HIPCHK(hipStreamWaitEvent(x, rs.fork, 0));
            }
            std::vector<char> cb(nb, 1);
            std::vector<std::exception_ptr> errs(nb);
            auto run = [&](int b) {
                try {
                    HIPCHK(hipSetDevice(dev));
                    cb[b] = run_basis(b, Bn[b], xks[b], sub[b], rs.st[b]) ? 1 : 0;
                } catch (...) {
                    errs[b] = std::current_exception();
                }
            };
            {
                std::vector<std::thread> th;
                for (int b = 1; b < nb; ++b) th.emplace_back(run, b);
                run(0);
                for (auto& x : th) x.join();
            }
            for (int b = 0; b < nb; ++b) {
                HIPCHK(hipEventRecord(rs.ev[b], rs.st[b]));
                HIPCHK(hipStreamWaitEvent(s, rs.ev[b], 0));
            }
            HIPCHK(hipStreamSynchronize(s));
            for (auto& e : errs)
                if (e) std::rethrow_exception(e);
            for (int b = 0; b < nb; ++b) out.all_conv = out.all_conv && cb[b];
        }
    }
    out.rep[0].sigma_builds += sig0;
    if (!g_dry) finish_amplitudes(xd, nroots, o + v, out.rep, op.dyson_out, s);
    ws.release(mark0);
    return out;
}

}  // namespace adc3

// ===========================================================================
// C ABI
// ===========================================================================
using namespace adc3;

struct adc3_ctx {
    Ctx* c;
};

static int setup_impl(const double* eps_occ, const double* eps_vir, const double* B, int nocc, int nvir, int naux,
                      int level, int precision, int ladder, double smx, void* workspace, size_t ws_bytes,
                      hipStream_t stream, adc3_ctx** ctx_out);

#define API_BEGIN try {
#define API_END                                   \
    }                                             \
    catch (const Error& e) {                      \
        g_dry = false;                            \
        set_error(e.msg);                         \
        return e.status;                          \
    }                                             \
    catch (const std::exception& e) {             \
        g_dry = false;                            \
        set_error(e.what());                      \
        return ADC3_EINVAL;                       \
    }

extern "C" {

void adc3_default_opts(adc3_opts* o) {
    if (!o) return;
    o->level = 3;
    o->max_iter = 500;
    o->max_subspace = 0;
    o->fno_correction = 1;
    o->precision = 0;
    o->precond = 3;
    o->mlp_weights = nullptr;
    o->sigma_graphs = 0;
    o->ladder = 0;
    o->sm_x = 1.0;
    o->fno_mode = 0;
    o->fno_keep_frac = 0.0;
    o->init_guess = nullptr;
    o->n_guess = 0;
    o->vectors_out = nullptr;
    o->dyson_out = nullptr;
    o->lockstep = -1;
}

const char* adc3_last_error(void) { return g_msg.c_str(); }

static void check_dims(int nocc, int nvir, int naux) {
    if (nocc <= 0 || nvir <= 0 || naux < 0) fail(ADC3_EINVAL, "nocc and nvir must be > 0 and naux >= 0");
    if (nvir > 1024) fail(ADC3_EINVAL, "nvir > 1024 is not supported");
}

size_t adc3_ea_setup_workspace_bytes_ex(int nocc, int nvir, int naux, int level, int nroots, int precision,
                                        int ladder) {
    try {
        check_dims(nocc, nvir, naux);
        if (level != 2 && level != 3) return 0;
        if (precision < 0 || precision > 2) return 0;
        if (ladder < 0 || ladder > 2) return 0;
        const bool df = ladder == 2 || (ladder == 0 && ladder_df_auto(nvir));
        Arena ws;
        g_dry = true;
        const long long n = nocc + nvir;
        take(ws, (long long)naux * n * n);  // split blocks of the public setup
        Ctx* c = build_ctx(ws, dry_vec(), dry_vec(), dry_vec(), dry_vec(), dry_vec(), nocc, nvir, naux, level, nullptr, precision,
                           df);
        {
            Arena w2 = ws;
            take(w2, 2LL * NVMAX * c->N);  // dense-matrix hook
            sigma_impl(c, w2, dry_vec(), dry_vec(), NVMAX, nullptr, precision);
            ws.peak = std::max(ws.peak, w2.peak);
        }
        if (nroots > 0) {
            Arena w3 = ws;
            take(w3, (long long)std::min<long long>(nroots, c->N) * c->N);  // converged vectors of adc3_mlp_collect
            davidson_impl(c, w3, (int)std::min<long long>(nroots, c->N), 1.0, 1, 0, nullptr, nullptr, precision);
            ws.peak = std::max(ws.peak, w3.peak);
        }
        delete c;
        g_dry = false;
        return ws.peak + (1 << 20);
    } catch (...) {
        g_dry = false;
        return 0;
    }
}

size_t adc3_ea_setup_workspace_bytes(int nocc, int nvir, int naux, int level, int nroots, int precision) {
    return adc3_ea_setup_workspace_bytes_ex(nocc, nvir, naux, level, nroots, precision, 0);
}

int adc3_ea_setup_ex(const double* eps_occ, const double* eps_vir, const double* B, int nocc, int nvir, int naux,
                     int level, int precision, int ladder, void* workspace, size_t ws_bytes, hipStream_t stream,
                     adc3_ctx** ctx_out) {
    API_BEGIN
    return setup_impl(eps_occ, eps_vir, B, nocc, nvir, naux, level, precision, ladder, 1.0, workspace, ws_bytes,
                      stream, ctx_out);
    API_END
}

}  // extern "C"

static int setup_impl(const double* eps_occ, const double* eps_vir, const double* B, int nocc, int nvir, int naux,
                      int level, int precision, int ladder, double smx, void* workspace, size_t ws_bytes,
                      hipStream_t stream, adc3_ctx** ctx_out) {
    {
    if (!ctx_out) fail(ADC3_EINVAL, "ctx_out is NULL");
    *ctx_out = nullptr;
    check_dims(nocc, nvir, naux);
    if (level != 2 && level != 3) fail(ADC3_EINVAL, "level must be 2 or 3");
    if (precision < 0 || precision > 2) fail(ADC3_EINVAL, "precision must be 0, 1 or 2");
    if (ladder < 0 || ladder > 2) fail(ADC3_EINVAL, "ladder must be 0 (auto), 1 (stored) or 2 (assembled)");
    const bool df = ladder == 2 || (ladder == 0 && ladder_df_auto(nvir));
    if (!eps_occ || !eps_vir || (!B && naux > 0) || !workspace) fail(ADC3_EINVAL, "NULL pointer argument");
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    const long long n = nocc + nvir;
    // split the factor into blocks (temporary, at the top of the workspace)
    const size_t mark0 = ws.mark();
    double* Boo = take(ws, (long long)naux * nocc * nocc);
    double* Bov = take(ws, (long long)naux * nocc * nvir);
    double* Bvv = take(ws, (long long)naux * nvir * nvir);
    k_split_B(B, naux, nocc, nvir, Boo, Bov, Bvv, stream);
    (void)n;
    Ctx* c = build_ctx(ws, eps_occ, eps_vir, Boo, Bov, Bvv, nocc, nvir, naux, level, stream, precision, df, smx);
    (void)mark0;
    HIPCHK(hipStreamSynchronize(stream));
    adc3_ctx* h = new adc3_ctx{c};
    *ctx_out = h;
    return ADC3_OK;
    }
}

extern "C" {

int adc3_ea_setup_sm(const double* eps_occ, const double* eps_vir, const double* B, int nocc, int nvir, int naux,
                     double sm_x, int precision, int ladder, void* workspace, size_t ws_bytes, hipStream_t stream,
                     adc3_ctx** ctx_out) {
    API_BEGIN
    if (!(sm_x >= 0.0 && sm_x <= 1.0)) fail(ADC3_EINVAL, "sm_x must lie in [0, 1]");
    return setup_impl(eps_occ, eps_vir, B, nocc, nvir, naux, 3, precision, ladder, sm_x, workspace, ws_bytes, stream,
                      ctx_out);
    API_END
}

int adc3_ea_setup(const double* eps_occ, const double* eps_vir, const double* B, int nocc, int nvir, int naux,
                  int level, int precision, void* workspace, size_t ws_bytes, hipStream_t stream, adc3_ctx** ctx_out) {
    return adc3_ea_setup_ex(eps_occ, eps_vir, B, nocc, nvir, naux, level, precision, 0, workspace, ws_bytes, stream,
                            ctx_out);
}

void adc3_ctx_destroy(adc3_ctx* ctx) {
    if (!ctx) return;
    delete ctx->c;
    delete ctx;
}

long long adc3_ea_dim(const adc3_ctx* ctx) { return ctx ? ctx->c->N : 0; }

int adc3_ea_sigma(adc3_ctx* ctx, const double* r, double* sigma, int nvec, int precision, hipStream_t stream) {
    API_BEGIN
    if (!ctx || !r || !sigma) fail(ADC3_EINVAL, "NULL argument");
    if (nvec < 0) fail(ADC3_EINVAL, "nvec < 0");
    if (precision != 0 && precision != ctx->c->prec)
        fail(ADC3_EINVAL, "precision must be 0 (FP64) or the context's setup precision");
    Arena ws = ctx->c->ws;
    sigma_impl(ctx->c, ws, r, sigma, nvec, stream, precision);
    return ADC3_OK;
    API_END
}

int adc3_ea_diagonal(adc3_ctx* ctx, double* diag, hipStream_t stream) {
    API_BEGIN
    if (!ctx || !diag) fail(ADC3_EINVAL, "NULL argument");
    k_copy(diag, ctx->c->diag, ctx->c->N, stream);
    return ADC3_OK;
    API_END
}

int adc3_ea_davidson(adc3_ctx* ctx, int nroots, double conv, int max_iter, int max_subspace, int precision,
                     double* omega, double* vectors, double* resnorm, int* iters, hipStream_t stream) {
    return adc3_ea_davidson_guess(ctx, nroots, conv, max_iter, max_subspace, precision, nullptr, 0, omega, vectors,
                                  resnorm, iters, stream);
}

int adc3_ea_davidson_guess(adc3_ctx* ctx, int nroots, double conv, int max_iter, int max_subspace, int precision,
                           const double* guess, int n_guess, double* omega, double* vectors, double* resnorm,
                           int* iters, hipStream_t stream) {
    API_BEGIN
    if (!ctx || !omega) fail(ADC3_EINVAL, "NULL argument");
    if (!(conv > 0)) fail(ADC3_EINVAL, "conv must be > 0");
    if (nroots < 1 || nroots > ctx->c->N) fail(ADC3_EINVAL, "nroots out of range");
    if (max_iter < 1) fail(ADC3_EINVAL, "max_iter must be >= 1");
    if (n_guess < 0 || (n_guess > 0 && !guess)) fail(ADC3_EINVAL, "n_guess > 0 needs guess vectors");
    if (precision != 0 && precision != ctx->c->prec)
        fail(ADC3_EINVAL, "precision must be 0 (FP64) or the context's setup precision");
    Arena ws = ctx->c->ws;
    DavResult r = davidson_impl(ctx->c, ws, nroots, conv, max_iter, max_subspace, vectors, stream, precision,
                                ctx->c->mlp_w != nullptr, nullptr, guess, n_guess);
    for (int k = 0; k < nroots; ++k) {
        omega[k] = r.w[k];
        if (resnorm) resnorm[k] = r.rn[k];
    }
    if (iters) *iters = r.iters;
    return r.converged ? ADC3_OK : ADC3_WNOCONV;
    API_END
}

int adc3_ea_dense_matrix(adc3_ctx* ctx, double* M, int ldm, hipStream_t stream) {
    API_BEGIN
    if (!ctx || !M) fail(ADC3_EINVAL, "NULL argument");
    const long long N = ctx->c->N;
    if (N > 20000) fail(ADC3_EINVAL, "dense matrix only for N <= 20000");
    if (ldm < N) fail(ADC3_EINVAL, "ldm < N");
    Arena ws = ctx->c->ws;
    double* E = take(ws, NVMAX * N);
    double* Sg = take(ws, NVMAX * N);
    std::vector<double> one(1, 1.0);
    for (long long j0 = 0; j0 < N; j0 += NVMAX) {
        int nb = (int)std::min<long long>(NVMAX, N - j0);
        k_fill(E, nb * N, 0.0, stream);
        for (int j = 0; j < nb; ++j) h2d(E + j * N + j0 + j, one.data(), sizeof(double), stream);
        sigma_impl(ctx->c, ws, E, Sg, nb, stream);
        // columns j0..j0+nb of M = rows of Sg (M symmetric)
        k_copy2d(M + j0 * ldm, ldm, Sg, N, nb, N, 1.0, 0.0, stream);
    }
    HIPCHK(hipStreamSynchronize(stream));
    return ADC3_OK;
    API_END
}

int adc3_ea_intermediate(adc3_ctx* ctx, int which, double* out, long long* count, hipStream_t stream) {
    API_BEGIN
    if (!ctx) fail(ADC3_EINVAL, "NULL ctx");
    Ctx* c = ctx->c;
    const long long vv = (long long)c->v * c->v;
    const double* src = nullptr;
    long long n = 0;
    switch (which) {
        case 0: src = c->M11; n = vv; break;
        case 1: src = c->Uz; n = vv * c->v * c->o; break;
        case 2: src = c->T; n = vv * c->o * c->o; break;
        case 3: src = c->Dmp2; n = vv; break;
        default: fail(ADC3_EINVAL, "unknown intermediate");
    }
    if (count) *count = n;
    if (out) k_copy(out, src, n, stream);
    return ADC3_OK;
    API_END
}

long long adc3_set_chunk_elems(long long n) {
    const long long prev = g_chunk_elems.load();
    if (n > 0) g_chunk_elems.store(n);
    return prev;
}

size_t adc3_ladder_workspace_bytes(int nvir, int naux, int nrows, int precision) {
    if (nvir <= 0 || naux < 0 || nrows <= 0 || precision < 0 || precision > 2) return 0;
    const size_t eb = precision == 0 ? 8 : precision == 1 ? 4 : 2;
    const size_t vv = (size_t)nvir * nvir;
    const size_t copies = precision == 0 ? 0 : (((size_t)naux * vv * eb + 255) & ~size_t(255)) + (((size_t)nrows * vv * eb + 255) & ~size_t(255));
    const size_t zt = precision == 2 ? ((size_t)nrows * vv + 8) * eb : 0;  // Z transposed (BF16)
    return copies + zt + (size_t)nrows * vv * eb;
}

int adc3_ladder_apply(const double* Bvv, const double* Z, double* C, int nvir, int naux, int nrows, int precision,
                      void* workspace, size_t ws_bytes, hipStream_t stream) {
    API_BEGIN
    if (nvir <= 0 || naux < 0 || nrows <= 0) fail(ADC3_EINVAL, "nvir and nrows must be > 0 and naux >= 0");
    if (nvir > 1024 || nrows > 65535) fail(ADC3_EINVAL, "nvir > 1024 or nrows > 65535 is not supported");
    if (precision < 0 || precision > 2) fail(ADC3_EINVAL, "precision must be 0, 1 or 2");
    if (!Bvv || !Z || !C || !workspace) fail(ADC3_EINVAL, "NULL pointer argument");
    const size_t need = adc3_ladder_workspace_bytes(nvir, naux, nrows, precision);
    if (ws_bytes < need) fail(ADC3_ENOMEM, "workspace too small: need at least " + std::to_string(need) + " bytes");
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    const long long vv = (long long)nvir * nvir;
    const void *Bp = Bvv, *Zp = Z;
    if (precision > 0) {
        void* Bl = precision == 1 ? (void*)ws.take<float>((size_t)std::max<long long>((long long)naux * vv, 1))
                                  : (void*)ws.take<unsigned short>((size_t)std::max<long long>((long long)naux * vv, 1));
        void* Zl = precision == 1 ? (void*)ws.take<float>((size_t)(nrows * vv))
                                  : (void*)ws.take<unsigned short>((size_t)(nrows * vv));
        k_to_lowp(Bl, Bvv, (long long)naux * vv, precision, stream);
        k_to_lowp(Zl, Z, nrows * vv, precision, stream);
        Bp = Bl;
        Zp = Zl;
    }
    const size_t eb = precision == 0 ? 8 : precision == 1 ? 4 : 2;
    const size_t off = (ws.used + 255) & ~size_t(255);
    const long long ve = (long long)((ws_bytes - std::min(ws_bytes, off)) / eb);
    if (ve < nrows * vv + (precision == 2 ? nrows * vv + 8 : 0))
        fail(ADC3_ENOMEM, "workspace too small for one auxiliary function of the intermediate");
    void* V = ws.base + off;
    const double fl = 4.0 * naux * (double)nrows * nvir * (double)vv;
    const double by = eb * (2.0 * naux * (double)nrows * vv + (double)naux * vv + nrows * (double)vv) + 8.0 * nrows * (double)vv;
    const double pk = precision == 0 ? PEAK_FP64_MFMA : precision == 1 ? PEAK_FP32_MFMA : PEAK_BF16_MFMA;
    ProfScope p(precision > 0 ? PROF_LADDER_LP : PROF_LADDER, stream, fl, by, 1e3 * std::max(fl / pk, by / PEAK_HBM));
    df_ladder(precision, nrows, nvir, naux, Bp, Zp, C, false, V, ve, stream);
    return ADC3_OK;
    API_END
}

size_t adc3_eigh_workspace_bytes(int n) {
    if (n <= 0 || n > 4096) return 0;
    return ((size_t)2 * n * n + eig_large_scratch(n) + n) * sizeof(double) + 4 * 256;
}

int adc3_eigh(const double* A, double* w, double* V, int n, void* workspace, size_t ws_bytes, hipStream_t stream) {
    API_BEGIN
    if (n <= 0 || n > 4096) fail(ADC3_EINVAL, "n must be in 1..4096");
    if (!A || !w || !V || !workspace) fail(ADC3_EINVAL, "NULL pointer argument");
    const size_t need = adc3_eigh_workspace_bytes(n);
    if (ws_bytes < need) fail(ADC3_ENOMEM, "workspace too small: need at least " + std::to_string(need) + " bytes");
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    const long long nn = (long long)n * n;
    double* Ac = take(ws, nn);
    double* scr = take(ws, (long long)eig_large_scratch(n));
    double* wt = take(ws, n);
    double* Vt = take(ws, nn);
    k_copy(Ac, A, nn, stream);
    k_symmetrize(Ac, n, stream);
    eig_large(Ac, n, w, V, scr, stream);
    k_sort_eig(w, V, n, 0, wt, Vt, stream);
    return ADC3_OK;
    API_END
}

size_t adc3_eigh_batched_workspace_bytes(int n, int nb) {
    if (n <= 0 || n > 4096 || nb <= 0 || nb > 65535) return 0;
    const size_t nn = (size_t)n * n;
    return ((size_t)nb * nn * 2 + eig_batched_scratch(n, nb) + n + nn + (size_t)nb * n) * sizeof(double) + 6 * 256;
}

int adc3_eigh_batched(const double* A, double* w, double* V, int n, int nb, void* workspace, size_t ws_bytes,
                      hipStream_t stream) {
    API_BEGIN
    if (n <= 0 || n > 4096 || nb <= 0 || nb > 65535) fail(ADC3_EINVAL, "n must be in 1..4096 and nb in 1..65535");
    if (!A || !w || !V || !workspace) fail(ADC3_EINVAL, "NULL pointer argument");
    const size_t need = adc3_eigh_batched_workspace_bytes(n, nb);
    if (ws_bytes < need) fail(ADC3_ENOMEM, "workspace too small: need at least " + std::to_string(need) + " bytes");
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    const long long nn = (long long)n * n;
    double* Ac = take(ws, nb * nn);
    double* Vu = take(ws, nb * nn);
    double* scr = take(ws, (long long)eig_batched_scratch(n, nb));
    double* wt = take(ws, n);
    double* Vt = take(ws, nn);
    k_copy(Ac, A, nb * nn, stream);
    for (int b = 0; b < nb; ++b) k_symmetrize(Ac + b * nn, n, stream);
    eig_batched(Ac, n, nb, w, Vu, scr, stream);
    for (int b = 0; b < nb; ++b) {
        k_sort_eig(w + (long long)b * n, Vu + b * nn, n, 0, wt, Vt, stream);
        k_copy(V + b * nn, Vu + b * nn, nn, stream);
    }
    return ADC3_OK;
    API_END
}

}  // extern "C"

static void validate_inputs(const double* eo, const double* ev, const double* B, int o, int v, int X, hipStream_t s,
                            Arena& ws) {
    std::vector<double> ho(o), hv(v);
    d2h(ho.data(), eo, o * sizeof(double), s);
    d2h(hv.data(), ev, v * sizeof(double), s);
    if (g_dry) return;
    for (int i = 0; i < o; ++i)
        if (!std::isfinite(ho[i]) || (i && ho[i] < ho[i - 1])) fail(ADC3_EINVAL, "eps_occ must be finite and ascending");
    for (int a = 0; a < v; ++a)
        if (!std::isfinite(hv[a]) || (a && hv[a] < hv[a - 1])) fail(ADC3_EINVAL, "eps_vir must be finite and ascending");
    if (!(ho[o - 1] < hv[0])) fail(ADC3_EINVAL, "every occupied energy must lie below every virtual energy");
    if (X > 0) {
        const size_t mark = ws.mark();
        double* f = take(ws, 4);
        k_check_B(B, X, o + v, f, s);
        unsigned long long hf[3];
        d2h(hf, f, sizeof(hf), s);
        double asym, mabs;
        std::memcpy(&asym, &hf[1], 8);
        std::memcpy(&mabs, &hf[2], 8);
        if (hf[0]) fail(ADC3_EINVAL, "B contains non-finite values");
        if (asym > 1e-12 * std::max(mabs, 1e-300)) fail(ADC3_EINVAL, "B must be symmetric in its orbital indices");
        ws.release(mark);
    }
}

static adc3_opts resolve_opts(const adc3_opts* opts) {
    adc3_opts o;
    adc3_default_opts(&o);
    if (opts) o = *opts;
    if (o.level != 2 && o.level != 3) fail(ADC3_EINVAL, "opts.level must be 2 or 3");
    if (o.max_iter < 1) fail(ADC3_EINVAL, "opts.max_iter must be >= 1");
    if (o.precision < 0 || o.precision > 2) fail(ADC3_EUNSUP, "opts.precision must be 0 (FP64), 1 (FP32) or 2 (BF16)");
    if (o.precond < 0 || o.precond > 3)
        fail(ADC3_EUNSUP, "opts.precond must be 0 (Jacobi), 1 (learned), 2 (Olsen) or 3 (exact 1p block)");
    if (o.precond == 1 && !o.mlp_weights) fail(ADC3_EINVAL, "opts.precond = 1 needs opts.mlp_weights");
    if (o.ladder < 0 || o.ladder > 2) fail(ADC3_EINVAL, "opts.ladder must be 0 (auto), 1 (stored) or 2 (assembled)");
    if (!(o.sm_x >= 0.0 && o.sm_x <= 1.0)) fail(ADC3_EINVAL, "opts.sm_x must lie in [0, 1]");
    if (o.fno_mode != 0 && o.fno_mode != 1) fail(ADC3_EINVAL, "opts.fno_mode must be 0 (state-specific) or 1 (MP2)");
    if (!(o.fno_keep_frac >= 0.0 && o.fno_keep_frac <= 1.0)) fail(ADC3_EINVAL, "opts.fno_keep_frac must lie in [0, 1]");
    if (o.n_guess < 0 || (o.n_guess > 0 && !o.init_guess)) fail(ADC3_EINVAL, "opts.n_guess > 0 needs opts.init_guess");
    if (o.lockstep < -1 || o.lockstep > 2) fail(ADC3_EINVAL, "opts.lockstep must be -1, 0, 1 or 2");
    return o;
}

// Workspace plan of one solve (a dry run with allocations counted): path 0 the canonical solve only,
// 1 the truncated pipeline only, 2 both (thresholds not known yet).
static void plan_solve(int nocc, int nvir, int naux, int nroots, const adc3_opts& op, Arena& ws, int path = 2) {
    g_dry = true;
    const long long n = nocc + nvir;
    Blocks B0;
    B0.X = naux; B0.o = nocc; B0.v = nvir;
    B0.Boo = take(ws, (long long)naux * nocc * nocc);
    B0.Bov = take(ws, (long long)naux * nocc * nvir);
    B0.Bvv = take(ws, (long long)naux * nvir * nvir);
    (void)n;
    adc3_opts oc = op;
    oc.fno_keep_frac = 0.0;  // the canonical path's plan must not take the truncated route
    if (path != 0) solve_impl(ws, dry_vec(), dry_vec(), B0, nroots, 1.0, 1.0, 1.0, op, nullptr);  // truncation path
    if (path != 1) {
        Arena ws2;
        ws2.used = 0;
        solve_impl(ws2, dry_vec(), dry_vec(), B0, nroots, 0.0, 0.0, 1.0, oc, nullptr);  // canonical path
        ws.peak = std::max(ws.peak, ws2.peak + (size_t)(3 * naux * n * n * sizeof(double)));
    }
    g_dry = false;
}

extern "C" size_t adc3_ea_solve_workspace_bytes(int nocc, int nvir, int naux, int nroots, const adc3_opts* opts) {
    try {
        check_dims(nocc, nvir, naux);
        adc3_opts op = resolve_opts(opts);
        Arena ws;
        plan_solve(nocc, nvir, naux, nroots, op, ws);
        return ws.peak + (1 << 20);
    } catch (...) {
        g_dry = false;
        return 0;
    }
}

// One instance: validate, split B, run the pipeline.  Throws Error; returns OK or WNOCONV.
static int solve_one(const double* eps_occ, const double* eps_vir, const double* B, int nocc, int nvir, int naux,
                     int nroots, double fno_thresh, double naf_thresh, double conv, const adc3_opts& op,
                     double* roots_out, adc3_root_report* reports, void* workspace, size_t ws_bytes,
                     hipStream_t stream) {
    check_dims(nocc, nvir, naux);
    if (!eps_occ || !eps_vir || (!B && naux > 0) || !roots_out || !workspace) fail(ADC3_EINVAL, "NULL pointer argument");
    const long long N = nvir + (long long)nocc * nvir * nvir;
    if (nroots < 1 || nroots > N) fail(ADC3_EINVAL, "nroots must be in [1, N]");
    if (!(conv > 0) || !std::isfinite(conv)) fail(ADC3_EINVAL, "conv must be a positive number");
    if (std::isnan(fno_thresh) || std::isnan(naf_thresh)) fail(ADC3_EINVAL, "thresholds must not be NaN");
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    {
        Arena plan;
        plan_solve(nocc, nvir, naux, nroots, op, plan, truncates(fno_thresh, naf_thresh, op) ? 1 : 0);
        if (plan.peak > ws_bytes) fail(ADC3_ENOMEM, "workspace too small: need " + std::to_string(plan.peak) + " bytes");
    }
    validate_inputs(eps_occ, eps_vir, B, nocc, nvir, naux, stream, ws);
    Blocks B0;
    B0.X = naux; B0.o = nocc; B0.v = nvir;
    B0.Boo = take(ws, (long long)naux * nocc * nocc);
    B0.Bov = take(ws, (long long)naux * nocc * nvir);
    B0.Bvv = take(ws, (long long)naux * nvir * nvir);
    k_split_B(B, naux, nocc, nvir, B0.Boo, B0.Bov, B0.Bvv, stream);
    SolveOut r = solve_impl(ws, eps_occ, eps_vir, B0, nroots, fno_thresh, naf_thresh, conv, op, stream);
    HIPCHK(hipStreamSynchronize(stream));
    for (int k = 0; k < nroots; ++k) {
        roots_out[k] = r.rep[k].omega;
        if (reports) reports[k] = r.rep[k];
    }
    return r.all_conv ? ADC3_OK : ADC3_WNOCONV;
}

extern "C" int adc3_ea_solve(const double* eps_occ, const double* eps_vir, const double* B, int nocc, int nvir,
                             int naux, int nroots, double fno_thresh, double naf_thresh, double conv,
                             const adc3_opts* opts, double* roots_out, adc3_root_report* reports, void* workspace,
                             size_t ws_bytes, hipStream_t stream) {
    API_BEGIN
    adc3_opts op = resolve_opts(opts);
    return solve_one(eps_occ, eps_vir, B, nocc, nvir, naux, nroots, fno_thresh, naf_thresh, conv, op, roots_out,
                     reports, workspace, ws_bytes, stream);
    API_END
}

// ---------------------------------------------------------------------------
// Ragged batches.  Instances are spread over worker streams (one host thread each) by
// longest-processing-time-first on an estimate of their work; a worker solves its
// instances in turn in its own slice of the workspace (sized for the largest of them).
// While one worker waits on a host synchronisation of its Davidson, the others keep
// the GPU busy, so small launch-bound instances overlap with each other and with the
// large ladder-bound ones.
// ---------------------------------------------------------------------------
namespace {
struct BatchPlan {
    std::vector<int> worker;        // per instance
    std::vector<size_t> offset;     // per worker, bytes into the workspace
    std::vector<size_t> bytes;      // per worker
    size_t total = 0;
};

double instance_cost(const adc3_instance& in) {
    const double o = in.nocc, v = in.nvir, X = in.naux, v4 = v * v * v * v;
    return 2.0 * o * v4 * in.nroots * 20.0 + 2.0 * X * v4 + 2.0 * o * o * v4 + 5e9;
}

BatchPlan plan_batch(const adc3_instance* inst, int ninst, const adc3_opts& op, int nworkers) {
    BatchPlan P;
    P.worker.assign(ninst, 0);
    std::vector<int> order(ninst);
    for (int i = 0; i < ninst; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return instance_cost(inst[a]) > instance_cost(inst[b]); });
    std::vector<double> load(nworkers, 0.0);
    P.bytes.assign(nworkers, 0);
    for (int i : order) {
        const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        P.worker[i] = w;
        load[w] += instance_cost(inst[i]);
        check_dims(inst[i].nocc, inst[i].nvir, inst[i].naux);
        Arena plan;
        plan_solve(inst[i].nocc, inst[i].nvir, inst[i].naux, inst[i].nroots, op, plan,
                   truncates(inst[i].fno_thresh, inst[i].naf_thresh, op) ? 1 : 0);
        P.bytes[w] = std::max(P.bytes[w], (plan.peak + (1 << 20) + 255) / 256 * 256);
    }
    P.offset.assign(nworkers, 0);
    for (int w = 0; w < nworkers; ++w) {
        P.offset[w] = P.total;
        P.total += P.bytes[w];
    }
    return P;
}

int batch_workers(int nstreams, int ninst) { return std::max(1, std::min(nstreams > 0 ? nstreams : 4, ninst)); }
}  // namespace

extern "C" size_t adc3_ea_solve_batched_workspace_bytes(const adc3_instance* inst, int ninst, const adc3_opts* opts,
                                                        int nstreams) {
    try {
        if (!inst || ninst < 1) return 0;
        adc3_opts op = resolve_opts(opts);
        return plan_batch(inst, ninst, op, batch_workers(nstreams, ninst)).total;
    } catch (...) {
        g_dry = false;
        return 0;
    }
}

// The batch in lockstep (opts.lockstep): waves of one instance per slot (each slot's instances in the
// plan's order, largest first), each wave's canonical solves built in their slots' workspace slices and
// their Davidsons advanced together by the lockstep engine on `stream`; an instance that truncates runs
// its own pipeline (its bases in lockstep) when its turn comes.  One host thread throughout.
static void batched_lockstep(const adc3_instance* inst, int ninst, const adc3_opts& op, const BatchPlan& P, int nw,
                             const std::vector<long long>& first, double* roots_out, adc3_root_report* reports,
                             std::vector<int>& st, std::vector<std::string>& msg, void* workspace, hipStream_t s) {
    std::vector<std::vector<int>> slot(nw);
    {
        std::vector<int> order(ninst);
        for (int i = 0; i < ninst; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return instance_cost(inst[a]) > instance_cost(inst[b]); });
        for (int i : order) slot[P.worker[i]].push_back(i);
    }
    size_t nwave = 0;
    for (auto& v : slot) nwave = std::max(nwave, v.size());
    struct SlotStreams {
        std::vector<hipStream_t> st;
        std::vector<hipEvent_t> ev;
        hipEvent_t wave = nullptr;
        ~SlotStreams() {
            if (wave) (void)hipEventDestroy(wave);
            for (auto e : ev) (void)hipEventDestroy(e);
            for (auto x : st) (void)hipStreamDestroy(x);
        }
    } slr;
    HIPCHK(hipEventCreateWithFlags(&slr.wave, hipEventDisableTiming));
    for (int sl = 0; sl < nw; ++sl) {
        hipStream_t x = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        slr.st.push_back(x);
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        slr.ev.push_back(e);
    }
    const std::vector<hipStream_t>& sls = slr.st;
    const std::vector<hipEvent_t>& sev = slr.ev;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    for (size_t w = 0; w < nwave; ++w) {
        // the slots' streams start after everything on the caller's stream: the inputs, and the previous
        // wave's work on the same workspace slices
        HIPCHK(hipEventRecord(slr.wave, s));
        for (int sl = 0; sl < nw; ++sl) HIPCHK(hipStreamWaitEvent(sls[sl], slr.wave, 0));
        std::vector<std::exception_ptr> errs(nw);
        std::vector<Arena> ar(nw);
        std::vector<Ctx*> ctx(nw, nullptr);
        std::vector<LockJob> jobs(nw);
        std::vector<double*> vecs(nw, nullptr);
        std::vector<size_t> jmark(nw, 0);  // each slot's arena before the lockstep buffers
        std::vector<int> who(nw, -1);
        std::vector<LockJob*> jp;
        // each slot's instance is checked and its context built on the slot's own stream by a host thread
        // of its own, so that the wave's setups overlap (an instance that truncates runs its whole pipeline
        // there); the wave's Davidsons then start together, ordered after every setup
        auto prepare = [&](int sl) {
            if (hipSetDevice(dev) != hipSuccess) {
                errs[sl] = std::make_exception_ptr(Error{ADC3_EHIP, "hipSetDevice failed in a slot thread"});
                return;
            }
            const int i = slot[sl][w];
            const adc3_instance& in = inst[i];
            hipStream_t ss = sls[sl];
            ar[sl].base = (char*)workspace + P.offset[sl];
            ar[sl].cap = P.bytes[sl];
            try {
                check_dims(in.nocc, in.nvir, in.naux);
                if (!in.eps_occ || !in.eps_vir || (!in.B && in.naux > 0)) fail(ADC3_EINVAL, "NULL pointer argument");
                const long long N = in.nvir + (long long)in.nocc * in.nvir * in.nvir;
                if (in.nroots < 1 || in.nroots > N) fail(ADC3_EINVAL, "nroots must be in [1, N]");
                if (!(in.conv > 0) || !std::isfinite(in.conv)) fail(ADC3_EINVAL, "conv must be a positive number");
                validate_inputs(in.eps_occ, in.eps_vir, in.B, in.nocc, in.nvir, in.naux, ss, ar[sl]);
                Blocks B0;
                B0.X = in.naux; B0.o = in.nocc; B0.v = in.nvir;
                B0.Boo = take(ar[sl], (long long)in.naux * in.nocc * in.nocc);
                B0.Bov = take(ar[sl], (long long)in.naux * in.nocc * in.nvir);
                B0.Bvv = take(ar[sl], (long long)in.naux * in.nvir * in.nvir);
                k_split_B(in.B, in.naux, in.nocc, in.nvir, B0.Boo, B0.Bov, B0.Bvv, ss);
                if (truncates(in.fno_thresh, in.naf_thresh, op)) {
                    SolveOut r = solve_impl(ar[sl], in.eps_occ, in.eps_vir, B0, in.nroots, in.fno_thresh,
                                            in.naf_thresh, in.conv, op, ss);
                    HIPCHK(hipStreamSynchronize(ss));
                    for (int k = 0; k < in.nroots; ++k) {
                        roots_out[first[i] + k] = r.rep[k].omega;
                        if (reports) reports[first[i] + k] = r.rep[k];
                    }
                    st[i] = r.all_conv ? ADC3_OK : ADC3_WNOCONV;
                    return;
                }
                const bool df = op.ladder == 2 || (op.ladder == 0 && ladder_df_auto(in.nvir));
                ctx[sl] = build_ctx(ar[sl], in.eps_occ, in.eps_vir, B0.Boo, B0.Bov, B0.Bvv, in.nocc, in.nvir, in.naux,
                                    op.level, ss, op.precision, df, op.level >= 3 ? op.sm_x : 1.0);
                vecs[sl] = take(ar[sl], (long long)in.nroots * N);
                jmark[sl] = ar[sl].mark();
                LockJob& j = jobs[sl];
                j.c = ctx[sl];
                j.nroots = in.nroots; j.conv = in.conv; j.max_iter = op.max_iter; j.max_sub = op.max_subspace;
                j.pmode = op.level >= 3 ? 0 : ((op.precond == 0) ? 0 : 3);
                j.prec = op.precision;
                j.vec_out = vecs[sl];
                j.arena = &ar[sl];
                who[sl] = i;
            } catch (const Error& e) {
                g_dry = false;
                st[i] = e.status;
                msg[i] = e.msg;
                if (ctx[sl]) { delete ctx[sl]; ctx[sl] = nullptr; }
                if (e.status == ADC3_EHIP) errs[sl] = std::current_exception();
            } catch (...) {
                if (ctx[sl]) { delete ctx[sl]; ctx[sl] = nullptr; }
                errs[sl] = std::current_exception();
            }
        };
        {
            std::vector<std::thread> th;
            for (int sl = 1; sl < nw; ++sl)
                if (w < slot[sl].size()) th.emplace_back(prepare, sl);
            if (w < slot[0].size()) prepare(0);
            for (auto& x : th) x.join();
        }
        for (auto& e : errs)
            if (e) std::rethrow_exception(e);
        for (int sl = 0; sl < nw; ++sl) {
            if (w >= slot[sl].size()) continue;
            HIPCHK(hipEventRecord(sev[sl], sls[sl]));
            HIPCHK(hipStreamWaitEvent(s, sev[sl], 0));
            if (who[sl] >= 0) jp.push_back(&jobs[sl]);
        }
        if (!jp.empty()) {
            try {
                lockstep_run(jp, s, lockstep_chunk());
                for (int sl = 0; sl < nw; ++sl) {
                    if (who[sl] < 0) continue;
                    const int i = who[sl];
                    const adc3_instance& in = inst[i];
                    const DavResult& r = jobs[sl].res;
                    std::vector<adc3_root_report> rep(in.nroots, adc3_root_report{});
                    const int o = in.nocc, v = in.nvir;
                    ar[sl].release(jmark[sl]);  // the Davidson's buffers (its vectors are in vecs)
                    GemmScratch gscr(ar[sl], GEMM_SCRATCH);
                    double* xd = take(ar[sl], (long long)in.nroots * (o + v));
                    double* tmp = take(ar[sl], (long long)o * v * v);
                    for (int k = 0; k < in.nroots; ++k) {
                        auto& R = rep[k];
                        R.omega = R.omega_uncorr = r.w[k];
                        R.omega_lowp = r.w_lowp.empty() ? r.w[k] : r.w_lowp[k];
                        R.iters_lowp = r.iters_lowp;
                        R.resnorm = R.err_bound = r.rn[k];
                        R.nvir_kept = v;
                        R.naux_kept = in.naux;
                        R.iters = r.iters;
                        R.sigma_builds = R.sigma_builds_final = k == 0 ? (int)jobs[sl].sigma_builds : 0;
                        spectral_amplitudes(ctx[sl], vecs[sl] + (long long)k * ctx[sl]->N, xd + (long long)k * (o + v),
                                            tmp, s);
                    }
                    finish_amplitudes(xd, in.nroots, o + v, rep, nullptr, s);
                    for (int k = 0; k < in.nroots; ++k) {
                        roots_out[first[i] + k] = rep[k].omega;
                        if (reports) reports[first[i] + k] = rep[k];
                    }
                    st[i] = r.converged ? ADC3_OK : ADC3_WNOCONV;
                }
            } catch (const Error& e) {
                g_dry = false;
                for (int sl = 0; sl < nw; ++sl)
                    if (who[sl] >= 0) { st[who[sl]] = e.status; msg[who[sl]] = e.msg; }
                if (e.status == ADC3_EHIP) {
                    for (auto* c : ctx) delete c;
                    throw;
                }
            }
        }
        for (auto* c : ctx) delete c;
    }
}

extern "C" int adc3_ea_solve_batched(const adc3_instance* inst, int ninst, const adc3_opts* opts, int nstreams,
                                     double* roots_out, adc3_root_report* reports, int* status_out, void* workspace,
                                     size_t ws_bytes, hipStream_t stream) {
    API_BEGIN
    if (!inst || ninst < 1 || !roots_out || !workspace) fail(ADC3_EINVAL, "NULL argument or ninst < 1");
    adc3_opts op = resolve_opts(opts);
    const int nw = batch_workers(nstreams, ninst);
    BatchPlan P = plan_batch(inst, ninst, op, nw);
    if (P.total > ws_bytes) fail(ADC3_ENOMEM, "workspace too small: need " + std::to_string(P.total) + " bytes");
    std::vector<long long> first(ninst + 1, 0);
    for (int i = 0; i < ninst; ++i) first[i + 1] = first[i] + std::max(inst[i].nroots, 0);
    if (op.lockstep == 1) {
        std::vector<int> st(ninst, ADC3_OK);
        std::vector<std::string> msg(ninst);
        batched_lockstep(inst, ninst, op, P, nw, first, roots_out, reports, st, msg, workspace, stream);
        int worst = ADC3_OK;
        std::string first_msg;
        for (int i = 0; i < ninst; ++i) {
            if (status_out) status_out[i] = st[i];
            if (st[i] < 0 && (worst >= 0 || st[i] < worst)) {
                if (first_msg.empty()) first_msg = "instance " + std::to_string(i) + ": " + msg[i];
                worst = st[i];
            } else if (st[i] == ADC3_WNOCONV && worst == ADC3_OK) {
                worst = ADC3_WNOCONV;
            }
        }
        if (worst < 0) set_error(first_msg);
        return worst;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    hipEvent_t ready;
    HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ready, stream));
    std::vector<int> st(ninst, ADC3_OK);
    std::vector<std::string> msg(ninst);
    std::vector<hipEvent_t> done(nw, nullptr);
    std::vector<std::thread> th;
    for (int w = 0; w < nw; ++w) {
        th.emplace_back([&, w]() {
            hipStream_t ws = nullptr;
            try {
                HIPCHK(hipSetDevice(dev));
                HIPCHK(hipStreamCreateWithFlags(&ws, hipStreamNonBlocking));
                HIPCHK(hipStreamWaitEvent(ws, ready, 0));
                for (int i = 0; i < ninst; ++i) {
                    if (P.worker[i] != w) continue;
                    try {
                        st[i] = solve_one(inst[i].eps_occ, inst[i].eps_vir, inst[i].B, inst[i].nocc, inst[i].nvir,
                                          inst[i].naux, inst[i].nroots, inst[i].fno_thresh, inst[i].naf_thresh,
                                          inst[i].conv, op, roots_out + first[i], reports ? reports + first[i] : nullptr,
                                          (char*)workspace + P.offset[w], P.bytes[w], ws);
                    } catch (const Error& e) {
                        g_dry = false;
                        st[i] = e.status;
                        msg[i] = e.msg;
                        if (e.status == ADC3_EHIP) break;  // the stream may be unusable
                    }
                }
                HIPCHK(hipEventCreateWithFlags(&done[w], hipEventDisableTiming));
                HIPCHK(hipEventRecord(done[w], ws));
                HIPCHK(hipStreamSynchronize(ws));
            } catch (const Error& e) {
                for (int i = 0; i < ninst; ++i)
                    if (P.worker[i] == w && st[i] == ADC3_OK) { st[i] = e.status; msg[i] = e.msg; }
            }
            if (ws) (void)hipStreamDestroy(ws);
        });
    }
    for (auto& t : th) t.join();
    for (int w = 0; w < nw; ++w)
        if (done[w]) {
            (void)hipStreamWaitEvent(stream, done[w], 0);
            (void)hipEventDestroy(done[w]);
        }
    (void)hipEventDestroy(ready);
    int worst = ADC3_OK;
    std::string first_msg;
    for (int i = 0; i < ninst; ++i) {
        if (status_out) status_out[i] = st[i];
        if (st[i] < 0 && (worst >= 0 || st[i] < worst)) {
            if (first_msg.empty()) first_msg = "instance " + std::to_string(i) + ": " + msg[i];
            worst = st[i];
        } else if (st[i] == ADC3_WNOCONV && worst == ADC3_OK) {
            worst = ADC3_WNOCONV;
        }
    }
    if (worst < 0) set_error(first_msg);
    return worst;
    API_END
}

extern "C" int adc3_ea_spectral_amplitudes(adc3_ctx* ctx, const double* vecs, int nvec, double* x,
                                           hipStream_t stream) {
    API_BEGIN
    if (!ctx || !vecs || !x) fail(ADC3_EINVAL, "NULL argument");
    if (nvec < 0) fail(ADC3_EINVAL, "nvec < 0");
    Ctx* c = ctx->c;
    Arena ws = c->ws;
    double* tmp = take(ws, (long long)c->o * c->v * c->v);
    for (int k = 0; k < nvec; ++k)
        spectral_amplitudes(c, vecs + (long long)k * c->N, x + (long long)k * (c->o + c->v), tmp, stream);
    return ADC3_OK;
    API_END
}

extern "C" void adc3_debug_inject_nan(int iteration) { g_nan_at.store(std::max(iteration, 0)); }

extern "C" int adc3_ea_set_sigma_graphs(adc3_ctx* ctx, int on) {
    API_BEGIN
    if (!ctx) fail(ADC3_EINVAL, "NULL ctx");
    ctx->c->graphs = on != 0;
    return ADC3_OK;
    API_END
}

extern "C" int adc3_mlp_nparams(void) { return mlp_nparam(); }

extern "C" int adc3_ea_set_preconditioner(adc3_ctx* ctx, const float* weights) {
    API_BEGIN
    if (!ctx) fail(ADC3_EINVAL, "NULL ctx");
    ctx->c->mlp_w = weights;
    return ADC3_OK;
    API_END
}

extern "C" int adc3_mlp_collect(adc3_ctx* ctx, int nroots, double conv, int max_iter, int group_size, int max_groups,
                                unsigned long long seed, double* feat, double* a0, double* target, int* ngroups,
                                hipStream_t stream) {
    API_BEGIN
    if (!ctx || !feat || !a0 || !target || !ngroups) fail(ADC3_EINVAL, "NULL argument");
    if (group_size < 1 || max_groups < 0) fail(ADC3_EINVAL, "group_size must be >= 1 and max_groups >= 0");
    if (!(conv > 0)) fail(ADC3_EINVAL, "conv must be > 0");
    if (nroots < 1 || nroots > ctx->c->N) fail(ADC3_EINVAL, "nroots out of range");
    Arena ws = ctx->c->ws;
    double* xf = take(ws, (long long)nroots * ctx->c->N);
    // pass 1: converged vectors; pass 2 replays the same (deterministic) solve and records
    DavResult r = davidson_impl(ctx->c, ws, nroots, conv, max_iter, 0, xf, stream, 0, false, nullptr);
    Recorder rec;
    rec.S = group_size; rec.Gmax = max_groups; rec.seed = seed; rec.xf = xf;
    rec.F = feat; rec.A0 = a0; rec.D = target;
    davidson_impl(ctx->c, ws, nroots, conv, max_iter, 0, nullptr, stream, 0, false, &rec);
    *ngroups = rec.G;
    return r.converged ? ADC3_OK : ADC3_WNOCONV;
    API_END
}

extern "C" size_t adc3_mlp_workspace_bytes(int batch_groups, int group_size) {
    const long long n = (long long)batch_groups * group_size;
    if (n <= 0) return 0;
    return (mlp_scratch_elems(n) + 3 * (size_t)n + 6 * (size_t)n + 4 * (size_t)mlp_nparam() + GEMM_SCRATCH + 4096) *
           sizeof(double) + (1 << 20);
}

extern "C" int adc3_mlp_loss_grad(const float* weights, const double* feat, const double* a0, const double* target,
                                  int ngroups, int group_size, double* grad, double* loss, void* workspace,
                                  size_t ws_bytes, hipStream_t stream) {
    API_BEGIN
    if (!weights || !feat || !a0 || !target || !loss || !workspace) fail(ADC3_EINVAL, "NULL argument");
    if (ngroups < 1 || group_size < 1) fail(ADC3_EINVAL, "ngroups and group_size must be >= 1");
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    const long long n = (long long)ngroups * group_size;
    double* scr = take(ws, (long long)mlp_scratch_elems(n));
    GemmScratch gscr(ws, GEMM_SCRATCH);
    *loss = mlp_loss_grad(weights, feat, a0, target, ngroups, group_size, grad, scr, nullptr, stream);
    return ADC3_OK;
    API_END
}

extern "C" int adc3_mlp_forward(const float* weights, const double* feat, long long n, double* u, void* workspace,
                                size_t ws_bytes, hipStream_t stream) {
    API_BEGIN
    if (!weights || !feat || !u || !workspace) fail(ADC3_EINVAL, "NULL argument");
    if (n < 1) fail(ADC3_EINVAL, "n must be >= 1");
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    double* H = take(ws, 4 * n * 256);
    GemmScratch gscr(ws, GEMM_SCRATCH);
    mlp_forward(weights, feat, n, u, H, H + n * 256, H + 2 * n * 256, H + 3 * n * 256, stream);
    HIPCHK(hipStreamSynchronize(stream));
    return ADC3_OK;
    API_END
}

extern "C" int adc3_mlp_train(float* weights, const double* feat, const double* a0, const double* target, int ngroups,
                              int group_size, int epochs, int batch_groups, double lr, unsigned long long seed,
                              double* loss_per_epoch, void* workspace, size_t ws_bytes, hipStream_t stream) {
    API_BEGIN
    if (!weights || !feat || !a0 || !target || !workspace) fail(ADC3_EINVAL, "NULL argument");
    if (ngroups < 1 || group_size < 1 || epochs < 1 || batch_groups < 1) fail(ADC3_EINVAL, "sizes must be >= 1");
    batch_groups = std::min(batch_groups, ngroups);
    Arena ws;
    ws.base = (char*)workspace;
    ws.cap = ws_bytes;
    const int S = group_size;
    const long long n = (long long)batch_groups * S;
    const int P = mlp_nparam();
    double* scr = take(ws, (long long)mlp_scratch_elems(n));
    double* bF = take(ws, n * 6);
    double* bA = take(ws, n);
    double* bD = take(ws, n);
    double* grad = take(ws, P);
    double* mom = take(ws, P);
    double* var = take(ws, P);
    GemmScratch gscr(ws, GEMM_SCRATCH);
    k_fill(mom, P, 0.0, stream);
    k_fill(var, P, 0.0, stream);
    // deterministic shuffles (splitmix64 on the host)
    unsigned long long st = seed;
    auto next = [&]() {
        unsigned long long z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    std::vector<int> order(ngroups);
    int step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int g = 0; g < ngroups; ++g) order[g] = g;
        for (int g = ngroups - 1; g > 0; --g) std::swap(order[g], order[(int)(next() % (unsigned long long)(g + 1))]);
        double lsum = 0.0;
        int nb = 0;
        for (int b0 = 0; b0 + batch_groups <= ngroups; b0 += batch_groups) {
            for (int j = 0; j < batch_groups; ++j) {
                const long long src = (long long)order[b0 + j] * S;
                k_copy(bF + (long long)j * S * 6, feat + src * 6, (long long)S * 6, stream);
                k_copy(bA + (long long)j * S, a0 + src, S, stream);
                k_copy(bD + (long long)j * S, target + src, S, stream);
            }
            lsum += mlp_loss_grad(weights, bF, bA, bD, batch_groups, S, grad, scr, nullptr, stream);
            mlp_adam(weights, grad, mom, var, lr, ++step, stream);
            ++nb;
        }
        if (loss_per_epoch) loss_per_epoch[ep] = nb ? lsum / nb : 0.0;
    }
    HIPCHK(hipStreamSynchronize(stream));
    return ADC3_OK;
    API_END
}

extern "C" int adc3_ea_precondition(adc3_ctx* ctx, double theta, const double* r, double* t, int* fallback,
                                    hipStream_t stream) {
    API_BEGIN
    if (!ctx || !r || !t) fail(ADC3_EINVAL, "NULL argument");
    Ctx* c = ctx->c;
    Arena ws = c->ws;
    unsigned int* flag = (unsigned int*)take(ws, 1);
    double* th = take(ws, 1);
    int fb = 0;
    if (c->mlp_w) {
        double* part = take(ws, (long long)dots_partial_elems(1, 1, c->N));
        k_dots(r, c->N, 1, r, c->N, 1, c->N, th, 1, part, stream);
        double nrm2 = 0;
        d2h(&nrm2, th, sizeof(double), stream);
        const double rms = std::max(std::sqrt(nrm2 / (double)c->N), 1e-300);
        HIPCHK(hipMemsetAsync(flag, 0, sizeof(unsigned int), stream));
        mlp_weights_bf16(c->mlp_w, c->mlp_wb, stream);
        mlp_precondition(r, c->diag, theta, rms, c->eo, c->ev, c->o, c->v, c->N, c->mlp_w, c->mlp_wb, t, flag, stream);
        unsigned int hf = 0;
        d2h(&hf, flag, sizeof(hf), stream);
        fb = hf != 0;
    } else {
        h2d(th, &theta, sizeof(double), stream);
        k_precond(t, r, c->diag, th, 1, c->N, stream);
    }
    HIPCHK(hipStreamSynchronize(stream));
    if (fallback) *fallback = fb;
    return ADC3_OK;
    API_END
}
