// Batched CPU engine: simultaneous multithreading over mini-batches plus SIMD inside each
// mini-batch, the paper's stronger CPU solver (Sec. 3.1: the batch is transposed into
// mini-batches whose instances sit side by side, one SIMD lane each; Sec. 4.2, Alg. 2: the
// left-looking refactorization with fixed pre-order and pattern, one mini-batch per
// thread; no column-level parallelism on the CPU).
//
// It executes the plan pf_analyze built for the GPU path (the same pre-order, L+U pattern,
// update lists with direct relative targets, and Jacobian position map), as the paper's
// three engines share one initialisation.  Every array of a mini-batch is stored
// element-major, instance-minor ([element][W]), so each inner loop is a W-wide vector
// operation.  A mini-batch runs the whole Newton loop; instances that have stopped keep
// their lane but no longer update their voltages.  This engine is a CPU baseline beside
// the GPU kernels, never a fallback for them.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "pf_internal.h"

namespace pf {

namespace {

constexpr int W = 8;   // instances per mini-batch: one 512-bit or two 256-bit FP64 vectors

// sin and cos of W angles: Cody-Waite reduction by pi/2 (three-part constant, fused
// multiply-adds), Taylor series of sin (to r^17) and cos (to r^18) on |r| <= pi/4, quadrant
// by the reduction count.  Written as straight-line lane loops so that they vectorise.
inline void sincos_w(const double *x, double *sn, double *cs)
{
    constexpr double two_over_pi = 0x1.45f306dc9c883p-1;
    constexpr double c1 = 0x1.921fb54442d18p+0, c2 = 0x1.1a62633145c07p-54, c3 = -0x1.f1976b7ed8fbcp-110;
    for (int b = 0; b < W; b++) {
        const double k = std::nearbyint(x[b] * two_over_pi);
        double r = std::fma(-k, c1, x[b]);
        r = std::fma(-k, c2, r);
        r = std::fma(-k, c3, r);
        const double r2 = r * r;
        double ps = 2.8114572543455206e-15;
        ps = std::fma(ps, r2, -7.647163731819816e-13);
        ps = std::fma(ps, r2, 1.6059043836821613e-10);
        ps = std::fma(ps, r2, -2.505210838544172e-08);
        ps = std::fma(ps, r2, 2.7557319223985893e-06);
        ps = std::fma(ps, r2, -0.0001984126984126984);
        ps = std::fma(ps, r2, 0.008333333333333333);
        ps = std::fma(ps, r2, -0.16666666666666666);
        const double s = std::fma(r * r2, ps, r);
        double pc = -1.5619206968586225e-16;
        pc = std::fma(pc, r2, 4.779477332387385e-14);
        pc = std::fma(pc, r2, -1.1470745597729725e-11);
        pc = std::fma(pc, r2, 2.08767569878681e-09);
        pc = std::fma(pc, r2, -2.755731922398589e-07);
        pc = std::fma(pc, r2, 2.48015873015873e-05);
        pc = std::fma(pc, r2, -0.001388888888888889);
        pc = std::fma(pc, r2, 0.041666666666666664);
        pc = std::fma(pc, r2, -0.5);
        const double c = std::fma(r2, pc, 1.0);
        const long long kq = (long long)std::fmin(std::fmax(k, -0x1p52), 0x1p52);
        const int q = (int)(kq & 3);
        const double so = (q & 1) ? c : s, co = (q & 1) ? s : c;
        sn[b] = (q & 2) ? -so : so;
        cs[b] = ((q + 1) & 2) ? -co : co;
    }
}

// Per-plan tables the engine derives once: the fill positions of L+U-I (zeroed before the
// Jacobian is written), and for every update (k -> j) the storage index of L(j, k), the
// entry that carries the forward substitution y_j -= L(j, k) y_k along (-1 if absent).
struct CpuTables {
    std::vector<int32_t> fill;
    std::vector<int32_t> fs_at;
};

void build_tables(const HostPlan &h, CpuTables &t)
{
    const int nnz = h.col_ptr[h.N];
    t.fill.clear();
    for (int e = 0; e < nnz; e++)
        if (!h.isj[e]) t.fill.push_back(e);
    t.fs_at.assign(h.upd.size(), -1);
    for (int j = 0; j < h.N; j++)
        for (int u = h.upd_ptr[j]; u < h.upd_ptr[j + 1]; u++) {
            const Update &up = h.upd[u];
            const int lcnt = up.krel_lcnt >> 16;
            for (int e = 0; e < lcnt; e++)
                if (h.rel[up.roff + e] == h.col_diag[j]) { t.fs_at[u] = up.lbeg + e; break; }
        }
}

struct Scratch {
    std::vector<double> vm, va, ps, qs, vr, vi, lu, y;
    void size(const HostPlan &h)
    {
        const size_t n = (size_t)h.n * W;
        vm.resize(n); va.resize(n); ps.resize(n); qs.resize(n); vr.resize(n); vi.resize(n);
        lu.resize((size_t)h.col_ptr[h.N] * W);
        y.resize((size_t)h.N * W);
    }
};

struct Job {
    const HostPlan *h;
    const CpuTables *t;
    const double *ybus, *sbus, *v0;
    double tol;
    int max_iter, batch;
    double *v_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    int8_t *status_out;
};

// The whole Newton loop of one mini-batch (instances b0 .. b0 + W - 1; lanes past the batch
// carry a copy of instance b0 and are discarded).
__attribute__((target_clones("arch=skylake-avx512", "arch=haswell", "default")))
void solve_minibatch(const Job &jb, Scratch &sc, int b0)
{
    const HostPlan &h = *jb.h;
    const CpuTables &tb = *jb.t;
    const int n = h.n, N = h.N;
    double *__restrict vm = sc.vm.data(), *__restrict va = sc.va.data();
    double *__restrict ps = sc.ps.data(), *__restrict qs = sc.qs.data();
    double *__restrict vr = sc.vr.data(), *__restrict vi = sc.vi.data();
    double *__restrict lu = sc.lu.data(), *__restrict y = sc.y.data();
    const double *yb = jb.ybus;

    // transpose to the mini-batch layout
    int lanes = std::min(W, jb.batch - b0);
    for (int i = 0; i < n; i++)
        for (int b = 0; b < W; b++) {
            const size_t o = ((size_t)(b0 + (b < lanes ? b : 0)) * n + i) * 2;
            vm[i * W + b] = jb.v0[o];
            va[i * W + b] = jb.v0[o + 1];
            ps[i * W + b] = jb.sbus[o];
            qs[i * W + b] = jb.sbus[o + 1];
        }
    int active[W], status[W], iters[W], nupd[W];
    for (int b = 0; b < W; b++) { active[b] = 1; status[b] = PF_ST_MAXITER; iters[b] = 0; nupd[b] = 0; }

    for (;;) {
        // ---- mismatch (Eq. 1, Alg. 1 sign) and the Jacobian written into its LU positions
        for (int i = 0; i < n; i++) sincos_w(va + (size_t)i * W, vi + (size_t)i * W, vr + (size_t)i * W);
        for (int i = 0; i < n; i++)
            for (int b = 0; b < W; b++) {
                vr[i * W + b] *= vm[i * W + b];
                vi[i * W + b] *= vm[i * W + b];
            }
        for (const int32_t e : tb.fill)
            for (int b = 0; b < W; b++) lu[(size_t)e * W + b] = 0.0;
        double mx[W], bad[W];
        for (int b = 0; b < W; b++) { mx[b] = 0.0; bad[b] = 0.0; }
        for (int i = 0; i < n; i++) {
            const double *Vr = vr + (size_t)i * W, *Vi = vi + (size_t)i * W;
            double ir[W], ii[W];
            for (int b = 0; b < W; b++) { ir[b] = 0.0; ii[b] = 0.0; }
            double ygr = 0.0, ygi = 0.0;
            int qdg = -1;
            for (int q = h.yrp[i]; q < h.yrp[i + 1]; q++) {
                const int k = h.yci[q];
                const double gr = yb[2 * q], gi = yb[2 * q + 1];
                const JPos jp = h.jpos[q];
                const double *Kr = vr + (size_t)k * W, *Ki = vi + (size_t)k * W, *Km = vm + (size_t)k * W;
                for (int b = 0; b < W; b++) {
                    const double cr = gr * Kr[b] - gi * Ki[b], ci = gr * Ki[b] + gi * Kr[b];   // Y_ik V_k
                    ir[b] += cr;
                    ii[b] += ci;
                    if (k != i) {
                        // w = V_i conj(Y_ik V_k): dS_i/dangle_k = -j w, dS_i/d|V_k| = w / |V_k|
                        const double wr = Vr[b] * cr + Vi[b] * ci, wi = Vi[b] * cr - Vr[b] * ci;
                        const double inv = 1.0 / Km[b];
                        if (jp.pt >= 0) lu[(size_t)jp.pt * W + b] = wi;
                        if (jp.pv >= 0) lu[(size_t)jp.pv * W + b] = wr * inv;
                        if (jp.qt >= 0) lu[(size_t)jp.qt * W + b] = -wr;
                        if (jp.qv >= 0) lu[(size_t)jp.qv * W + b] = wi * inv;
                    }
                }
                if (k == i) { ygr = gr; ygi = gi; qdg = q; }
            }
            const int pe = h.bus_peq[i], qe = h.bus_qeq[i];
            for (int b = 0; b < W; b++) {
                const double sr = Vr[b] * ir[b] + Vi[b] * ii[b], si = Vi[b] * ir[b] - Vr[b] * ii[b];   // S_i
                if (qdg >= 0) {
                    // dS_i/dangle_i = j (S_i - |V_i|^2 conj Y_ii), dS_i/d|V_i| = S_i/|V_i| + |V_i| conj Y_ii
                    const JPos jp = h.jpos[qdg];
                    const double m = vm[i * W + b], m2 = m * m;
                    if (jp.pt >= 0) lu[(size_t)jp.pt * W + b] = -si - m2 * ygi;
                    if (jp.pv >= 0) lu[(size_t)jp.pv * W + b] = sr / m + m * ygr;
                    if (jp.qt >= 0) lu[(size_t)jp.qt * W + b] = sr - m2 * ygr;
                    if (jp.qv >= 0) lu[(size_t)jp.qv * W + b] = si / m - m * ygi;
                }
                if (pe >= 0) {
                    const double f = sr - ps[i * W + b];
                    y[(size_t)pe * W + b] = f;
                    if (std::isfinite(f)) mx[b] = std::fmax(mx[b], std::fabs(f)); else bad[b] = 1.0;
                }
                if (qe >= 0) {
                    const double f = si - qs[i * W + b];
                    y[(size_t)qe * W + b] = f;
                    if (std::isfinite(f)) mx[b] = std::fmax(mx[b], std::fabs(f)); else bad[b] = 1.0;
                }
            }
        }
        // ---- convergence test (before every update, strictly below tol)
        int any = 0;
        for (int b = 0; b < W; b++) {
            if (!active[b]) continue;
            if (bad[b] != 0.0) { status[b] = PF_ST_NONFINITE; active[b] = 0; iters[b] = nupd[b]; }
            else if (mx[b] < jb.tol) { status[b] = PF_ST_CONVERGED; active[b] = 0; iters[b] = nupd[b]; }
            else if (nupd[b] >= jb.max_iter) { status[b] = PF_ST_MAXITER; active[b] = 0; iters[b] = nupd[b]; }
            any |= active[b];
        }
        if (!any) break;

        // ---- left-looking refactorization with the forward substitution carried along
        int piv[W];
        for (int b = 0; b < W; b++) piv[b] = 0;
        for (int j = 0; j < N; j++) {
            double *col = lu + (size_t)h.col_ptr[j] * W;
            double *yj = y + (size_t)j * W;
            const int cnt = h.col_ptr[j + 1] - h.col_ptr[j];
            // largest magnitude of the column of A, for the relative pivot test
            double cmax[W];
            for (int b = 0; b < W; b++) cmax[b] = 0.0;
            for (int e = 0; e < cnt; e++)
                for (int b = 0; b < W; b++) cmax[b] = std::fmax(cmax[b], std::fabs(col[(size_t)e * W + b]));
            for (int u = h.upd_ptr[j]; u < h.upd_ptr[j + 1]; u++) {
                const Update &up = h.upd[u];
                const int krel = up.krel_lcnt & 0xffff, lcnt = up.krel_lcnt >> 16;
                const double *m = col + (size_t)krel * W;
                const double *src = lu + (size_t)up.lbeg * W;
                const int32_t *rel = h.rel.data() + up.roff;
                for (int e = 0; e < lcnt; e++) {
                    double *dst = col + (size_t)rel[e] * W;
                    const double *l = src + (size_t)e * W;
                    for (int b = 0; b < W; b++) dst[b] = std::fma(-m[b], l[b], dst[b]);
                }
                if (tb.fs_at[u] >= 0) {
                    const double *ljk = lu + (size_t)tb.fs_at[u] * W;
                    const double *yk = y + (size_t)up.k * W;
                    for (int b = 0; b < W; b++) yj[b] = std::fma(-ljk[b], yk[b], yj[b]);
                }
            }
            const int dr = h.col_diag[j];
            const double *d = col + (size_t)dr * W;
            // a pivot that is not finite, not above 1e-300 or below 1e-14 of its column's
            // largest magnitude fails the instance (as on the GPU)
            for (int b = 0; b < W; b++)
                if (!(std::fabs(d[b]) > 1e-300 && std::isfinite(d[b]) && std::fabs(d[b]) >= 1e-14 * cmax[b])) piv[b] = 1;
            for (int e = dr + 1; e < cnt; e++)
                for (int b = 0; b < W; b++) col[(size_t)e * W + b] /= d[b];
        }
        // ---- back substitution z_j = (y_j - sum_i U(j, i) z_i) / U(j, j), then V <- V - z
        for (int j = N - 1; j >= 0; j--) {
            double acc[W];
            for (int b = 0; b < W; b++) acc[b] = 0.0;
            for (int q = h.bs_ptr[j]; q < h.bs_ptr[j + 1]; q++) {
                const double *u = lu + (size_t)h.bs_pos[q] * W;
                const double *z = y + (size_t)h.bs_col[q] * W;
                for (int b = 0; b < W; b++) acc[b] = std::fma(u[b], z[b], acc[b]);
            }
            const double *d = lu + (size_t)(h.col_ptr[j] + h.col_diag[j]) * W;
            double *yj = y + (size_t)j * W;
            for (int b = 0; b < W; b++) yj[b] = (yj[b] - acc[b]) / d[b];
        }
        for (int b = 0; b < W; b++)
            if (active[b] && piv[b]) { status[b] = PF_ST_PIVOT; active[b] = 0; iters[b] = nupd[b]; }
        for (int j = 0; j < N; j++) {
            const int pu = h.pos_upd[j];
            double *tgt = ((pu & 1) ? vm : va) + (size_t)(pu >> 1) * W;
            const double *z = y + (size_t)j * W;
            for (int b = 0; b < W; b++)
                if (active[b]) tgt[b] -= z[b];
        }
        for (int b = 0; b < W; b++) nupd[b] += active[b];
    }

    for (int b = 0; b < lanes; b++) {
        const int g = b0 + b;
        for (int i = 0; i < n; i++) {
            jb.v_out[((size_t)g * n + i) * 2] = vm[i * W + b];
            jb.v_out[((size_t)g * n + i) * 2 + 1] = va[i * W + b];
        }
        jb.iters_out[g] = iters[b];
        jb.conv_out[g] = status[b] == PF_ST_CONVERGED ? 1 : 0;
        if (jb.status_out) jb.status_out[g] = (int8_t)status[b];
    }
}

}  // namespace

int cpu_solve(const HostPlan &h, int32_t batch, const double *ybus, const double *sbus, const double *v0, double tol,
              int32_t max_iter, int32_t threads, double *v_out, int32_t *iters_out, uint8_t *conv_out,
              int8_t *status_out, std::string &err)
{
    CpuTables tb;
    try {
        build_tables(h, tb);
    } catch (const std::bad_alloc &) {
        err = "out of host memory";
        return PF_ENOMEM;
    }
    Job jb{&h, &tb, ybus, sbus, v0, tol, max_iter, batch, v_out, iters_out, conv_out, status_out};
    const int nmb = (batch + W - 1) / W;
    int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::max(1, std::min(nt, nmb));
    std::atomic<int> next{0};
    std::atomic<int> failed{0};
    auto work = [&]() {
        Scratch sc;
        try {
            sc.size(h);
        } catch (const std::bad_alloc &) {
            failed = 1;
            return;
        }
        for (int m; (m = next.fetch_add(1)) < nmb;) solve_minibatch(jb, sc, m * W);
    };
    std::vector<std::thread> pool;
    try {
        for (int t = 1; t < nt; t++) pool.emplace_back(work);
    } catch (const std::exception &) {
        // fewer threads than asked: the calling thread and those started do the work
    }
    work();
    for (auto &th : pool) th.join();
    if (failed) { err = "out of host memory for a mini-batch's scratch"; return PF_ENOMEM; }
    return PF_OK;
}

}  // namespace pf
