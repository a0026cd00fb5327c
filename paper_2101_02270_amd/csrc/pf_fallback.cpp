// Second chance for instances whose refactorization failed.  The paper checks the
// mismatch of every task on the CPU and solves a task that could not converge because of
// numerical trouble in the LU refactorization once more with a pivoting numerical
// factorization (Sec. 3.2, the KLU second chance; Sec. 4.1: partial pivoting updates the
// row permutation of Eq. 3 so that no tiny pivot is used).  The GPU path refactorizes with
// the fixed symmetric pre-order and diagonal pivots and flags such instances
// (PF_ST_PIVOT, or PF_ST_NONFINITE when a bad step made the mismatch non-finite); this file
// re-solves exactly those instances on the host:
//
//   * Newton-Raphson in FP64 from the instance's own start (Sec. 3: mismatch Eq. 1,
//     analytic polar Jacobian Sec. 3.1.2, V <- V - dx), the same stopping rules as the GPU
//     path;
//   * each Newton system A dx' = F' (A = P J P^T in the plan's pre-order, the Jacobian
//     written through the plan's position map) is factorized from scratch by a
//     left-looking Gilbert-Peierls LU with threshold partial pivoting: the column's
//     structure comes from a depth-first search over the columns of L already computed
//     (so fill follows the pivots), and the pivot row is the diagonal one when its
//     magnitude is at least kPivotThreshold times the largest candidate, otherwise the
//     largest candidate.
//
// The entry points are pf_cpu_solve_pivoting (host arrays, any batch) and
// pf_solve_fallback (device arrays of a pf_solve_batch call: only the flagged instances
// are copied to the host, solved and written back).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "pf_internal.h"

using namespace pf;

namespace {

constexpr double kPivotThreshold = 0.1;   // diagonal kept while |a_jj| >= 0.1 max |a_ij|

// A = P L U with row pivoting; L unit lower (by columns, original row indices, pivot row
// excluded), U upper (by columns, pivot-step indices, diagonal last).
struct PivotingLU {
    int N = 0;
    std::vector<int> lp, li, up, ui;
    std::vector<double> lx, ux;
    std::vector<int> row_of_step, step_of_row;   // pivot step -> original row and back (-1)
    // work arrays of the factorization
    std::vector<double> x;
    std::vector<int> mark, stack, child, reach, pattern;

    void reset(int n)
    {
        N = n;
        lp.assign(1, 0); up.assign(1, 0);
        li.clear(); lx.clear(); ui.clear(); ux.clear();
        row_of_step.assign(n, -1);
        step_of_row.assign(n, -1);
        x.assign(n, 0.0);
        mark.assign(n, -1);
        stack.resize(n); child.resize(n);
        reach.clear(); pattern.clear();
    }

    // Factorizes the CSC matrix (cp, ri, v) of order N.  Returns false when a column has
    // no usable pivot (all candidates zero or non-finite).
    bool factor(const std::vector<int> &cp, const std::vector<int> &ri, const std::vector<double> &v)
    {
        for (int j = 0; j < N; j++) {
            // structure of column j of L^-1 A: rows reachable from A(:, j) through the
            // columns of L computed so far; `reach` collects pivot steps in reverse
            // topological order (a step after every step it depends on when read backwards)
            reach.clear();
            pattern.clear();
            for (int e = cp[j]; e < cp[j + 1]; e++) {
                const int r0 = ri[e];
                if (mark[r0] == j) continue;
                // iterative depth-first search from r0
                int depth = 0;
                stack[0] = r0;
                mark[r0] = j;
                child[0] = -1;
                while (depth >= 0) {
                    const int r = stack[depth];
                    const int k = step_of_row[r];
                    int &c = child[depth];
                    if (c < 0) c = k >= 0 ? lp[k] : 0;
                    bool pushed = false;
                    if (k >= 0)
                        while (c < lp[k + 1]) {
                            const int r2 = li[c++];
                            if (mark[r2] != j) {
                                mark[r2] = j;
                                stack[++depth] = r2;
                                child[depth] = -1;
                                pushed = true;
                                break;
                            }
                        }
                    if (pushed) continue;
                    pattern.push_back(r);
                    if (k >= 0) reach.push_back(k);
                    depth--;
                }
            }
            for (int e = cp[j]; e < cp[j + 1]; e++) x[ri[e]] = v[e];
            // sparse triangular solve in topological order
            for (int a = (int)reach.size() - 1; a >= 0; a--) {
                const int k = reach[a];
                const double xk = x[row_of_step[k]];
                if (xk == 0.0) continue;
                for (int c = lp[k]; c < lp[k + 1]; c++) x[li[c]] -= lx[c] * xk;
            }
            // U(:, j): the pivotal rows, in ascending step order, then the pivot
            std::vector<std::pair<int, double>> ucol;
            ucol.reserve(reach.size());
            for (const int k : reach) ucol.emplace_back(k, x[row_of_step[k]]);
            std::sort(ucol.begin(), ucol.end());
            // pivot among the rows not yet pivotal
            double amax = 0.0;
            int pmax = -1;
            bool finite = true;
            for (const int r : pattern)
                if (step_of_row[r] < 0) {
                    const double a = std::fabs(x[r]);
                    if (!std::isfinite(a)) finite = false;
                    if (a > amax) { amax = a; pmax = r; }
                }
            int piv = pmax;
            if (step_of_row[j] < 0 && mark[j] == j && std::fabs(x[j]) >= kPivotThreshold * amax && x[j] != 0.0)
                piv = j;
            if (!finite || piv < 0 || amax == 0.0) {
                for (const int r : pattern) x[r] = 0.0;
                return false;
            }
            const double d = x[piv];
            for (const auto &kv : ucol) { ui.push_back(kv.first); ux.push_back(kv.second); }
            ui.push_back(j);
            ux.push_back(d);
            up.push_back((int)ui.size());
            for (const int r : pattern)
                if (step_of_row[r] < 0 && r != piv && x[r] != 0.0) { li.push_back(r); lx.push_back(x[r] / d); }
            lp.push_back((int)li.size());
            row_of_step[j] = piv;
            step_of_row[piv] = j;
            for (const int r : pattern) x[r] = 0.0;
        }
        return true;
    }

    // Solves A z = b (b indexed by original row, z by column); b is overwritten.
    void solve(std::vector<double> &b, std::vector<double> &z) const
    {
        for (int k = 0; k < N; k++) {
            const double yk = b[row_of_step[k]];
            z[k] = yk;
            if (yk != 0.0)
                for (int c = lp[k]; c < lp[k + 1]; c++) b[li[c]] -= lx[c] * yk;
        }
        for (int j = N - 1; j >= 0; j--) {
            const int last = up[j + 1] - 1;      // the diagonal
            const double zj = z[j] / ux[last];
            z[j] = zj;
            for (int c = up[j]; c < last; c++) z[ui[c]] -= ux[c] * zj;
        }
    }
};

// Scratch of one worker: Jacobian values in the plan's L+U storage, the extracted CSC
// matrix of A, right-hand side and step.
struct Work {
    std::vector<double> vm, va, vr, vi, lu, f, dx;
    std::vector<int> cp, ri;
    std::vector<double> av;
    PivotingLU lu_p;
};

// The Newton loop of one instance with a fresh pivoting factorization per iteration.
void solve_one(const HostPlan &h, const double *ybus, const double *sbus, const double *v0, double tol,
               int max_iter, double *v_out, int32_t &iters, uint8_t &conv, int8_t &status, Work &w)
{
    const int n = h.n, N = h.N;
    const int nnz = h.col_ptr[N];
    w.vm.resize(n); w.va.resize(n); w.vr.resize(n); w.vi.resize(n);
    w.lu.assign(nnz, 0.0);
    w.f.resize(N); w.dx.resize(N);
    for (int i = 0; i < n; i++) { w.vm[i] = v0[2 * i]; w.va[i] = v0[2 * i + 1]; }
    // the pattern of A without fill (fill entries hold no Jacobian value)
    w.cp.assign(N + 1, 0);
    w.ri.clear();
    for (int j = 0; j < N; j++) {
        for (int e = h.col_ptr[j]; e < h.col_ptr[j + 1]; e++)
            if (h.isj[e]) w.ri.push_back(h.row_idx[e]);
        w.cp[j + 1] = (int)w.ri.size();
    }
    w.av.resize(w.ri.size());
    int nupd = 0;
    for (;;) {
        for (int i = 0; i < n; i++) {
            w.vr[i] = w.vm[i] * std::cos(w.va[i]);
            w.vi[i] = w.vm[i] * std::sin(w.va[i]);
        }
        double mx = 0.0;
        bool bad = false;
        for (int i = 0; i < n; i++) {
            double ir = 0.0, ii = 0.0, ygr = 0.0, ygi = 0.0;
            int qdg = -1;
            for (int q = h.yrp[i]; q < h.yrp[i + 1]; q++) {
                const int k = h.yci[q];
                const double gr = ybus[2 * q], gi = ybus[2 * q + 1];
                const double cr = gr * w.vr[k] - gi * w.vi[k], ci = gr * w.vi[k] + gi * w.vr[k];   // Y_ik V_k
                ir += cr;
                ii += ci;
                if (k == i) { ygr = gr; ygi = gi; qdg = q; continue; }
                // w = V_i conj(Y_ik V_k): dS_i/dangle_k = -j w, dS_i/d|V_k| = w / |V_k|
                const double wr = w.vr[i] * cr + w.vi[i] * ci, wi = w.vi[i] * cr - w.vr[i] * ci;
                const JPos jp = h.jpos[q];
                if (jp.pt >= 0) w.lu[jp.pt] = wi;
                if (jp.pv >= 0) w.lu[jp.pv] = wr / w.vm[k];
                if (jp.qt >= 0) w.lu[jp.qt] = -wr;
                if (jp.qv >= 0) w.lu[jp.qv] = wi / w.vm[k];
            }
            const double sr = w.vr[i] * ir + w.vi[i] * ii, si = w.vi[i] * ir - w.vr[i] * ii;     // S_i
            if (qdg >= 0) {
                const JPos jp = h.jpos[qdg];
                const double m = w.vm[i], m2 = m * m;
                if (jp.pt >= 0) w.lu[jp.pt] = -si - m2 * ygi;
                if (jp.pv >= 0) w.lu[jp.pv] = sr / m + m * ygr;
                if (jp.qt >= 0) w.lu[jp.qt] = sr - m2 * ygr;
                if (jp.qv >= 0) w.lu[jp.qv] = si / m - m * ygi;
            }
            const double fp = sr - sbus[2 * i], fq = si - sbus[2 * i + 1];
            if (h.bus_peq[i] >= 0) {
                w.f[h.bus_peq[i]] = fp;
                if (std::isfinite(fp)) mx = std::fmax(mx, std::fabs(fp)); else bad = true;
            }
            if (h.bus_qeq[i] >= 0) {
                w.f[h.bus_qeq[i]] = fq;
                if (std::isfinite(fq)) mx = std::fmax(mx, std::fabs(fq)); else bad = true;
            }
        }
        if (bad) { status = PF_ST_NONFINITE; break; }
        if (mx < tol) { status = PF_ST_CONVERGED; break; }
        if (nupd >= max_iter) { status = PF_ST_MAXITER; break; }
        for (int j = 0, a = 0; j < N; j++)
            for (int e = h.col_ptr[j]; e < h.col_ptr[j + 1]; e++)
                if (h.isj[e]) w.av[a++] = w.lu[e];
        w.lu_p.reset(N);
        if (!w.lu_p.factor(w.cp, w.ri, w.av)) { status = PF_ST_PIVOT; break; }
        w.lu_p.solve(w.f, w.dx);
        for (int j = 0; j < N; j++) {
            const int pu = h.pos_upd[j];
            double &tgt = (pu & 1) ? w.vm[pu >> 1] : w.va[pu >> 1];
            tgt -= w.dx[j];
        }
        nupd++;
    }
    iters = nupd;
    conv = status == PF_ST_CONVERGED ? 1 : 0;
    for (int i = 0; i < n; i++) { v_out[2 * i] = w.vm[i]; v_out[2 * i + 1] = w.va[i]; }
}

// Solves the instances idx[0 .. count) of host arrays on `threads` workers.
int solve_list(const HostPlan &h, const int32_t *idx, int count, const double *ybus, size_t ybus_stride,
               const double *sbus, const double *v0, double tol, int max_iter, int threads, double *v_out,
               int32_t *iters_out, uint8_t *conv_out, int8_t *status_out, std::string &err)
{
    int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
    nt = std::max(1, std::min(nt, count));
    std::atomic<int> next{0}, failed{0};
    const size_t vs = (size_t)2 * h.n;
    auto work = [&]() {
        try {
            Work w;
            for (int a; (a = next.fetch_add(1)) < count;) {
                const int b = idx ? idx[a] : a;
                int8_t st = 0;
                solve_one(h, ybus + ybus_stride * b, sbus + vs * b, v0 + vs * b, tol, max_iter, v_out + vs * b,
                          iters_out[b], conv_out[b], st, w);
                if (status_out) status_out[b] = st;
            }
        } catch (const std::bad_alloc &) {
            failed = 1;
        }
    };
    std::vector<std::thread> pool;
    try {
        for (int t = 1; t < nt; t++) pool.emplace_back(work);
    } catch (const std::exception &) {
    }
    work();
    for (auto &th : pool) th.join();
    if (failed) { err = "out of host memory"; return PF_ENOMEM; }
    return PF_OK;
}

}  // namespace

extern "C" {

int pf_cpu_solve_pivoting(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched, const double *sbus,
                          const double *v0, double tol, int32_t max_iter, int32_t threads, double *v_out,
                          int32_t *iters_out, uint8_t *converged_out, int8_t *status_out)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl) { set_error("null plan"); return PF_EINVAL; }
    if (batch < 0 || threads < 0) { set_error("negative batch or thread count"); return PF_EINVAL; }
    if (batch == 0) return PF_OK;
    if (!ybus || !sbus || !v0 || !v_out || !iters_out || !converged_out) { set_error("null pointer"); return PF_EINVAL; }
    if (max_iter < 0 || !(tol >= 0.0)) { set_error("invalid tol or max_iter"); return PF_EINVAL; }
    std::string err;
    const int rc = solve_list(pl->h, nullptr, batch, ybus, ybus_batched ? (size_t)2 * pl->h.nnzy : 0, sbus, v0, tol,
                              max_iter, threads, v_out, iters_out, converged_out, status_out, err);
    if (rc != PF_OK) set_error(err);
    return rc;
}

int pf_solve_fallback(pf_plan plan, int32_t batch, const double *ybus, int32_t ybus_batched, const double *sbus,
                      const double *v0, double tol, int32_t max_iter, int32_t threads, double *v_out,
                      int32_t *iters_out, uint8_t *converged_out, int8_t *status_out, int32_t *n_resolved,
                      void *stream)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl) { set_error("null plan"); return PF_EINVAL; }
    if (batch < 0 || threads < 0) { set_error("negative batch or thread count"); return PF_EINVAL; }
    if (n_resolved) *n_resolved = 0;
    if (batch == 0) return PF_OK;
    if (!ybus || !sbus || !v0 || !v_out || !iters_out || !converged_out || !status_out) {
        set_error("null pointer (status_out is required)");
        return PF_EINVAL;
    }
    if (max_iter < 0 || !(tol >= 0.0)) { set_error("invalid tol or max_iter"); return PF_EINVAL; }
    const HostPlan &h = pl->h;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    auto fail = [&](const char *what, hipError_t e) {
        set_error(std::string(what) + ": " + hipGetErrorString(e));
        return PF_EDEVICE;
    };
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail("stream synchronisation failed", e);
    std::vector<int8_t> status(batch);
    if ((e = hipMemcpy(status.data(), status_out, batch, hipMemcpyDeviceToHost)) != hipSuccess)
        return fail("status copy failed", e);
    std::vector<int32_t> idx;
    for (int b = 0; b < batch; b++)
        if (status[b] == PF_ST_PIVOT || status[b] == PF_ST_NONFINITE) idx.push_back(b);
    if (idx.empty()) return PF_OK;
    const int m = (int)idx.size();
    const size_t vs = (size_t)2 * h.n, ys = (size_t)2 * h.nnzy;
    // the flagged instances' inputs, packed
    std::vector<double> y(ybus_batched ? ys * m : ys), s(vs * m), v(vs * m), vo(vs * m);
    std::vector<int32_t> it(m);
    std::vector<uint8_t> cv(m);
    std::vector<int8_t> so(m);
    if (!ybus_batched && (e = hipMemcpy(y.data(), ybus, ys * 8, hipMemcpyDeviceToHost)) != hipSuccess)
        return fail("ybus copy failed", e);
    for (int a = 0; a < m; a++) {
        const size_t b = idx[a];
        if ((e = hipMemcpy(s.data() + vs * a, sbus + vs * b, vs * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
            (e = hipMemcpy(v.data() + vs * a, v0 + vs * b, vs * 8, hipMemcpyDeviceToHost)) != hipSuccess ||
            (ybus_batched &&
             (e = hipMemcpy(y.data() + ys * a, ybus + ys * b, ys * 8, hipMemcpyDeviceToHost)) != hipSuccess))
            return fail("input copy failed", e);
    }
    std::string err;
    const int rc = solve_list(h, nullptr, m, y.data(), ybus_batched ? ys : 0, s.data(), v.data(), tol, max_iter,
                              threads, vo.data(), it.data(), cv.data(), so.data(), err);
    if (rc != PF_OK) { set_error(err); return rc; }
    for (int a = 0; a < m; a++) {
        const size_t b = idx[a];
        if ((e = hipMemcpy(v_out + vs * b, vo.data() + vs * a, vs * 8, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(iters_out + b, &it[a], 4, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(converged_out + b, &cv[a], 1, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(status_out + b, &so[a], 1, hipMemcpyHostToDevice)) != hipSuccess)
            return fail("result copy failed", e);
    }
    if (n_resolved) *n_resolved = m;
    return PF_OK;
}

}  // extern "C"
