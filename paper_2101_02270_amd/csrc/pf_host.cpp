// Solve of a host-resident batch with transfers overlapped with compute: the batch is cut
// into chunks, and two streams alternate copy-in, solve and copy-out, so chunk i+1's
// inputs travel over PCIe while chunk i is solved (the paper overlaps its host-device
// transfers with kernels through streams, Sec. 2.2 and Sec. 5.3).  Built on the public
// entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>

#include "pf_internal.h"

using namespace pf;

namespace {

struct HostRun {
    hipStream_t st[2] = {nullptr, nullptr};
    hipEvent_t start = nullptr, fin[2] = {nullptr, nullptr};
    void *dev = nullptr;
    ~HostRun()
    {
        for (int i = 0; i < 2; i++) {
            if (st[i]) (void)hipStreamDestroy(st[i]);
            if (fin[i]) (void)hipEventDestroy(fin[i]);
        }
        if (start) (void)hipEventDestroy(start);
        if (dev) (void)hipFree(dev);
    }
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" int pf_solve_host(pf_plan plan, int32_t batch, const double *ybus, const double *sbus_host,
                             const double *v0_host, double tol, int32_t max_iter, const pf_solve_opts *opts,
                             int32_t chunk, double *v_out_host, int32_t *iters_host, uint8_t *converged_host,
                             int8_t *status_host, void *stream)
{
    Plan *pl = reinterpret_cast<Plan *>(plan);
    if (!pl) { set_error("null plan"); return PF_EINVAL; }
    if (batch < 0 || chunk <= 0) { set_error("batch must be >= 0 and chunk > 0"); return PF_EINVAL; }
    if (batch == 0) return PF_OK;
    if (!ybus || !sbus_host || !v0_host || !v_out_host || !iters_host || !converged_host) {
        set_error("null pointer");
        return PF_EINVAL;
    }
    const int32_t cb = std::min(chunk, batch);
    const size_t n = (size_t)pl->h.n;
    pf_solve_opts o{};
    if (opts) o = *opts;
    // one configuration for every chunk, chosen for the chunk size
    if (pf_resolve_opts(plan, cb, &o, &o) != PF_OK) return PF_EINVAL;
    const size_t ws = pf_workspace_bytes(plan, cb, &o);
    if (ws == 0) return PF_EINVAL;
    const size_t vb = sizeof(double) * 2 * n * cb;
    // per stream: sbus, v0, v_out, iters, converged, status, workspace
    const size_t per = a256(vb) * 3 + a256(sizeof(int32_t) * cb) + a256((size_t)cb) * 2 + a256(ws);
    HostRun r;
    if (hipMalloc(&r.dev, 2 * per) != hipSuccess) {
        (void)hipGetLastError();
        r.dev = nullptr;
        set_error("out of device memory for the pipelined solve");
        return PF_ENOMEM;
    }
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; i++) {
        e = hipStreamCreateWithFlags(&r.st[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&r.fin[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r.start, hipEventDisableTiming);
    // the chunks start after the work already queued on the caller's stream
    if (e == hipSuccess) e = hipEventRecord(r.start, reinterpret_cast<hipStream_t>(stream));
    for (int i = 0; i < 2 && e == hipSuccess; i++) e = hipStreamWaitEvent(r.st[i], r.start, 0);
    if (e != hipSuccess) { set_error(std::string("stream setup failed: ") + hipGetErrorString(e)); return PF_EDEVICE; }

    int rc = PF_OK;
    for (int32_t b0 = 0, c = 0; b0 < batch && rc == PF_OK; b0 += cb, c++) {
        const int32_t m = std::min(cb, batch - b0);
        hipStream_t st = r.st[c & 1];
        char *p = static_cast<char *>(r.dev) + (size_t)(c & 1) * per;
        double *d_s = reinterpret_cast<double *>(p);
        double *d_v0 = reinterpret_cast<double *>(p + a256(vb));
        double *d_v = reinterpret_cast<double *>(p + 2 * a256(vb));
        int32_t *d_it = reinterpret_cast<int32_t *>(p + 3 * a256(vb));
        uint8_t *d_cv = reinterpret_cast<uint8_t *>(p + 3 * a256(vb) + a256(sizeof(int32_t) * cb));
        int8_t *d_st = reinterpret_cast<int8_t *>(d_cv + a256((size_t)cb));
        void *d_ws = d_st + a256((size_t)cb);
        const size_t off = (size_t)b0 * 2 * n, bytes = sizeof(double) * 2 * n * m;
        e = hipMemcpyAsync(d_s, sbus_host + off, bytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(d_v0, v0_host + off, bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) { set_error(std::string("copy-in failed: ") + hipGetErrorString(e)); rc = PF_EDEVICE; break; }
        rc = pf_solve_batch(plan, m, ybus, 0, d_s, d_v0, tol, max_iter, &o, d_ws, ws, d_v, d_it, d_cv, d_st, st);
        if (rc != PF_OK) break;
        e = hipMemcpyAsync(v_out_host + off, d_v, bytes, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(iters_host + b0, d_it, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(converged_host + b0, d_cv, (size_t)m, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && status_host)
            e = hipMemcpyAsync(status_host + b0, d_st, (size_t)m, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) { set_error(std::string("copy-out failed: ") + hipGetErrorString(e)); rc = PF_EDEVICE; }
    }
    // wait for both streams (also after an error: the buffers are freed on return)
    for (int i = 0; i < 2; i++) {
        if (hipStreamSynchronize(r.st[i]) != hipSuccess && rc == PF_OK) {
            set_error("pipelined solve failed on the device");
            rc = PF_EDEVICE;
        }
    }
    return rc;
}
