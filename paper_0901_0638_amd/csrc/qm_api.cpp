/*
 * qm_api.cpp -- the C ABI of libqm (include/qm.h): argument validation,
 * context, per-nu and per-(alpha, beta, delta) table caches, and dispatch
 * to the kernels.
 */
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "qm_batch.h"
#include "qm_context.h"
#include "qm_serve.h"

namespace {

thread_local std::string g_last_error;

qm_status fail(qm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
qm_status fail(qm_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

qm_status hip_fail(hipError_t e, const char* what)
{
    return fail(QM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t dtype_size(int dtype) { return dtype == QM_F64 ? 8 : 4; }

static bool vg_params_ok(double lambda, double alpha, double beta)
{
    return std::isfinite(lambda) && std::isfinite(alpha) && std::isfinite(beta) && lambda >= 1 && lambda <= 8 &&
           alpha > std::fabs(beta);
}

bool mode_known(uint32_t m) { return m == QM_PLAIN || m == QM_F32_REFINE || m == QM_PAPER || m == QM_PAPER_T2; }

bool hyp_params_ok(double alpha, double beta, double delta)
{
    return std::isfinite(alpha) && std::isfinite(beta) && std::isfinite(delta) && delta > 0 && alpha > std::fabs(beta);
}

}  // namespace

namespace qm {

qm_status check_request(const qm_request& r, int* dtype_size_out, bool single_call)
{
    if (r.reserved != 0) return fail(QM_E_INVAL, "reserved field must be 0");
    if (r.dtype != QM_F32 && r.dtype != QM_F64) return fail(QM_E_INVAL, "unknown dtype %u", r.dtype);
    if (!mode_known(r.mode)) return fail(QM_E_INVAL, "unknown mode %u", r.mode);
    switch (r.kind) {
    case QM_NORMAL_QUANTILE:
        if (r.dtype == QM_F64 && r.mode == QM_F32_REFINE)
            return fail(QM_E_DTYPE, "QM_F32_REFINE needs dtype QM_F32");
        if (r.dtype == QM_F32 && r.mode == QM_PAPER_T2) return fail(QM_E_DTYPE, "QM_PAPER_T2 needs dtype QM_F64");
        /* its wave vote ties an element's path to the other elements of its
           wave, so it would break the batch's bitwise equality with the
           single call */
        if (r.mode == QM_PAPER_T2 && !single_call)
            return fail(QM_E_INVAL, "QM_PAPER_T2 is a qm_normal_quantile mode only");
        break;
    case QM_EXP_TO_NORMAL:
        if (r.mode == QM_PAPER_T2) return fail(QM_E_DTYPE, "QM_PAPER_T2 is for the normal quantile only");
        if (r.dtype == QM_F64 && r.mode == QM_F32_REFINE)
            return fail(QM_E_DTYPE, "QM_F32_REFINE needs dtype QM_F32");
        if (r.dtype == QM_F32 && r.mode == QM_PAPER)
            return fail(QM_E_DTYPE, "exp->normal in FP32: QM_F32_REFINE or QM_PLAIN");
        break;
    case QM_STUDENT_T:
        if (!(r.dtype == QM_F64 && r.mode == QM_PLAIN) && !(r.dtype == QM_F32 && r.mode == QM_F32_REFINE))
            return fail(QM_E_DTYPE, "Student t: F64 QM_PLAIN or F32 QM_F32_REFINE");
        if (std::isnan(r.nu) || !(r.nu >= qm::T_NU_MIN))
            return fail(QM_E_INVAL, "nu must be >= %g or +inf (got %g)", qm::T_NU_MIN, r.nu);
        break;
    case QM_EXP_TO_HYPERBOLIC:
        if (!(r.dtype == QM_F64 && r.mode == QM_PLAIN) && !(r.dtype == QM_F32 && r.mode == QM_F32_REFINE))
            return fail(QM_E_DTYPE, "exp->hyperbolic: F64 QM_PLAIN or F32 QM_F32_REFINE");
        if (!hyp_params_ok(r.alpha, r.beta, r.delta))
            return fail(QM_E_INVAL, "need |beta| < alpha, delta > 0, all finite (got %g, %g, %g)", r.alpha, r.beta,
                        r.delta);
        if (!std::isfinite(r.mu)) return fail(QM_E_INVAL, "mu must be finite");
        break;
    case QM_EXP_TO_VG:
        if (!(r.dtype == QM_F64 && r.mode == QM_PLAIN) && !(r.dtype == QM_F32 && r.mode == QM_F32_REFINE))
            return fail(QM_E_DTYPE, "exp->variance-gamma: F64 QM_PLAIN or F32 QM_F32_REFINE");
        if (!vg_params_ok(r.nu, r.alpha, r.beta))
            return fail(QM_E_INVAL, "need lambda in [1, 8] and |beta| < alpha, all finite (got %g, %g, %g)",
                        r.nu, r.alpha, r.beta);
        if (!std::isfinite(r.mu)) return fail(QM_E_INVAL, "mu must be finite");
        break;
    default:
        return fail(QM_E_INVAL, "unknown kind %u", r.kind);
    }
    size_t es = dtype_size(r.dtype);
    if (r.n > 0) {
        if (!r.d_in || !r.d_out) return fail(QM_E_INVAL, "NULL buffer with n > 0");
        uintptr_t a = (uintptr_t)r.d_in, b = (uintptr_t)r.d_out;
        if (a % es || b % es) return fail(QM_E_INVAL, "buffers must be aligned to the element size");
        if (r.n > (UINT64_MAX / 2) / es) return fail(QM_E_INVAL, "n too large");
        uint64_t bytes = r.n * es;
        if (a != b && a < b + bytes && b < a + bytes) return fail(QM_E_INVAL, "input and output partially overlap");
    }
    if (dtype_size_out) *dtype_size_out = (int)es;
    return QM_OK;
}

/* Look up (or build and upload) the table for nu.  The build runs outside
   the table lock, so lookups of other tables (the serving loop's) never
   wait for it; if two threads build the same table, the first insert wins. */
qm_status get_table(qm_ctx* ctx, double nu, const DeviceTable** out)
{
    {
        std::lock_guard<std::mutex> lk(ctx->table_mu);
        auto it = ctx->tables.find(nu);
        if (it != ctx->tables.end()) { *out = &it->second; return QM_OK; }
    }
    HostTTable ht{};
    char err[256] = {0};
    if (build_student_table(nu, &ht, err, sizeof err) != 0)
        return fail(QM_E_INVAL, "Student t table for nu=%g: %s", nu, err);
    size_t coef_bytes = (size_t)ht.ncoef * sizeof(double);
    size_t bytes = sizeof(TTableHeader) + coef_bytes;
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) { free_student_table(&ht); return fail(QM_E_NOMEM, "hipMalloc table: %s", hipGetErrorString(e)); }
    e = hipMemcpy(d, &ht.hdr, sizeof(TTableHeader), hipMemcpyHostToDevice);
    if (e == hipSuccess && coef_bytes)
        e = hipMemcpy((char*)d + sizeof(TTableHeader), ht.coef, coef_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(d); free_student_table(&ht); return hip_fail(e, "upload table"); }
    DeviceTable dt;
    dt.hdr = ht.hdr;
    dt.d_table = (TTableHeader*)d;
    free_student_table(&ht);
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto res = ctx->tables.emplace(nu, dt);
    if (!res.second) (void)hipFree(d);   /* another thread's copy is already in use */
    *out = &res.first->second;
    return QM_OK;
}

qm_status find_table(qm_ctx* ctx, double nu, const DeviceTable** out)
{
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto it = ctx->tables.find(nu);
    if (it == ctx->tables.end())
        return fail(QM_E_INVAL, "no Student t table for nu=%g in the context yet (one call with this nu, "
                                "even with n = 0, builds it)", nu);
    *out = &it->second;
    return QM_OK;
}

qm_status find_base_table(qm_ctx* ctx, bool vg, double p1, double p2, double p3, const DeviceHypTable** out)
{
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto& tables = vg ? ctx->vg_tables : ctx->hyp_tables;
    auto it = tables.find(std::make_tuple(p1, p2, p3));
    if (it == tables.end())
        return fail(QM_E_INVAL, "no %s table for (%g, %g, %g) in the context yet (one call with these parameters, "
                                "even with n = 0, builds it)", vg ? "variance-gamma" : "hyperbolic", p1, p2, p3);
    *out = &it->second;
    return QM_OK;
}

/* Look up (or build and upload) a table of the two-sided exponential base:
   hyperbolic for (alpha, beta, delta), or variance-gamma for (lambda, alpha,
   beta) when vg; built outside the lock like get_table's. */
static qm_status get_base_table(qm_ctx* ctx, bool vg, double p1, double p2, double p3, const DeviceHypTable** out)
{
    auto key = std::make_tuple(p1, p2, p3);
    auto& tables = vg ? ctx->vg_tables : ctx->hyp_tables;
    {
        std::lock_guard<std::mutex> lk(ctx->table_mu);
        auto it = tables.find(key);
        if (it != tables.end()) { *out = &it->second; return QM_OK; }
    }
    HostHypTable ht{};
    char err[256] = {0};
    if (vg ? build_vg_table(p1, p2, p3, &ht, err, sizeof err) != 0
           : build_hyperbolic_table(p1, p2, p3, &ht, err, sizeof err) != 0)
        return fail(QM_E_INVAL, "%s table for (%g, %g, %g): %s", vg ? "variance-gamma" : "hyperbolic", p1, p2, p3, err);
    size_t coef_bytes = (size_t)ht.ncoef * sizeof(double);
    void* d = nullptr;
    hipError_t e = hipMalloc(&d, sizeof(HypTableHeader) + coef_bytes);
    if (e != hipSuccess) { free_hyperbolic_table(&ht); return fail(QM_E_NOMEM, "hipMalloc table: %s", hipGetErrorString(e)); }
    e = hipMemcpy(d, &ht.hdr, sizeof(HypTableHeader), hipMemcpyHostToDevice);
    if (e == hipSuccess && coef_bytes)
        e = hipMemcpy((char*)d + sizeof(HypTableHeader), ht.coef, coef_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(d); free_hyperbolic_table(&ht); return hip_fail(e, "upload table"); }
    DeviceHypTable dt;
    dt.hdr = ht.hdr;
    dt.d_table = (HypTableHeader*)d;
    dt.ncoef = ht.ncoef;
    free_hyperbolic_table(&ht);
    std::lock_guard<std::mutex> lk(ctx->table_mu);
    auto res = tables.emplace(key, dt);
    if (!res.second) (void)hipFree(d);
    *out = &res.first->second;
    return QM_OK;
}

qm_status get_hyp_table(qm_ctx* ctx, double alpha, double beta, double delta, const DeviceHypTable** out)
{
    return get_base_table(ctx, false, alpha, beta, delta, out);
}

qm_status get_vg_table(qm_ctx* ctx, double lambda, double alpha, double beta, const DeviceHypTable** out)
{
    return get_base_table(ctx, true, lambda, alpha, beta, out);
}

const TTableHeader* device_table_ptr(const DeviceTable* t) { return t->d_table; }
const TTableHeader& device_table_hdr(const DeviceTable* t) { return t->hdr; }
const LaunchShape& ctx_shape(const qm_ctx* ctx) { return ctx->shape; }
int ctx_device(const qm_ctx* ctx) { return ctx->device; }
uint64_t ctx_budget(const qm_ctx* ctx) { return ctx->budget; }

qm_status run_single(qm_ctx* ctx, const qm_request& r, hipStream_t s)
{
    /* a table is built (and cached) even for n = 0, so that a call can
       prepare it ahead of time */
    hipError_t e;
    if (r.kind == QM_STUDENT_T) {
        const DeviceTable* t = nullptr;
        qm_status st = get_table(ctx, r.nu, &t);
        if (st != QM_OK || r.n == 0) return st;
        e = launch_student(r.dtype, r.mode, r.d_in, r.d_out, r.n, t->d_table, t->hdr, s, ctx->shape);
    } else if (r.kind == QM_EXP_TO_HYPERBOLIC || r.kind == QM_EXP_TO_VG) {
        const DeviceHypTable* t = nullptr;
        qm_status st = r.kind == QM_EXP_TO_VG ? get_vg_table(ctx, r.nu, r.alpha, r.beta, &t)
                                              : get_hyp_table(ctx, r.alpha, r.beta, r.delta, &t);
        if (st != QM_OK || r.n == 0) return st;
        e = launch_hyperbolic(r.dtype, r.mode, r.d_in, r.d_out, r.n, t->d_table, t->hdr, t->ncoef, r.mu, s,
                              ctx->shape);
    } else {
        if (r.n == 0) return QM_OK;
        e = launch_elementwise(r.kind, r.dtype, r.mode, r.d_in, r.d_out, r.n, s, ctx->shape);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QM_OK;
}

}  // namespace qm

extern "C" {

qm_status qm_init(int hip_device, uint64_t hbm_budget_bytes, qm_ctx** out)
{
    if (!out) return fail(QM_E_INVAL, "out is NULL");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (hip_device < 0 || hip_device >= count) return fail(QM_E_INVAL, "no HIP device %d (%d present)", hip_device, count);
    e = hipSetDevice(hip_device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    qm_ctx* c = new (std::nothrow) qm_ctx;
    if (!c) return fail(QM_E_NOMEM, "context allocation");
    c->device = hip_device;
    c->budget = hbm_budget_bytes;
    c->cus = cus > 0 ? cus : 256;
    /* launch shapes per kernel family (workgroups of 256 per CU x vectors
       per lane), the best of measured sweeps over 1..64 x 1..4 on MI355X;
       QM_BLOCKS_PER_CU / QM_UNROLL override every family (tuning) */
    const uint64_t ncu = (uint64_t)(cus > 0 ? cus : 256);
    struct { qm::KernelShape* ks; const char* env; long bpc, unroll; } fam[] = {
        {&c->shape.stream, "QM_SHAPE_STREAM", 2, 4},   /* light maps: few workgroups, deep unroll */
        /* FP32 maps: four elements per 16-byte vector carry twice the
           arithmetic per byte; exp -> normal FP32 (2^26, scrubbed launches)
           ran 473-478 Gs/s refined and 590-600 plain at 16..32 x 2, against
           393-411 and 498-526 at 2 x 4 */
        {&c->shape.stream32, "QM_SHAPE_STREAM32", 32, 2},
        /* quantiles, wave-contiguous tiles: FP32+refine 16 x 4 (8..16 x 4
           measured 0.504-0.505 ms on the 2^28 FP32 mixture, 32 x 2 0.52-0.54),
           FP64 64 x 4 */
        {&c->shape.hybrid[0], "QM_SHAPE_NQ32", 16, 4},
        {&c->shape.hybrid[1], "QM_SHAPE_NQ64", 64, 4},
        /* fused generation (grid-stride), FP32 and FP64 outputs */
        {&c->shape.generate[0], "QM_SHAPE_GEN32", 32, 2},
        {&c->shape.generate[1], "QM_SHAPE_GEN64", 64, 4},
        {&c->shape.student[0], "QM_SHAPE_T32", 3, 4},  /* Student t, FP32 outputs */
        {&c->shape.student[1], "QM_SHAPE_T64", 2, 4},  /* Student t, FP64 outputs */
        /* exp -> hyperbolic, FP32, wave-contiguous tiles: 16 x 2 (670 Gs/s on
           2^26 base samples; 645 at 6 x 2, 658-673 at 8..16 x 2..4) */
        {&c->shape.hyperbolic[0], "QM_SHAPE_H32", 16, 2},
        /* exp -> hyperbolic, FP64, wave-contiguous tiles: 16 x 4 (0.185-0.186
           ms on 2^26 base samples, against 0.189-0.199 at 4..8 x 2..4) */
        {&c->shape.hyperbolic[1], "QM_SHAPE_H64", 16, 4},
    };
    long env_bpc = 0, env_unroll = 0;
    if (const char* ev = getenv("QM_BLOCKS_PER_CU")) env_bpc = strtol(ev, nullptr, 10);
    if (const char* ev = getenv("QM_UNROLL")) env_unroll = strtol(ev, nullptr, 10);
    for (auto& f : fam) {
        long bpc = f.bpc, unroll = f.unroll, eb = env_bpc, eu = env_unroll;
        if (const char* ev = getenv(f.env)) {       /* "bpc,unroll" for this family alone */
            char* end = nullptr;
            eb = strtol(ev, &end, 10);
            eu = (end && *end == ',') ? strtol(end + 1, nullptr, 10) : 0;
        }
        if (eb >= 1 && eb <= 64) bpc = eb;
        if (eu == 1 || eu == 2 || eu == 4) unroll = eu;
        f.ks->max_blocks = ncu * (uint64_t)bpc;
        f.ks->unroll = (int)unroll;
    }
    const char* ec = getenv("QM_COMPACT");
    c->shape.compact = ec ? (int)strtol(ec, nullptr, 10) != 0 : 1;
    /* set-up of the allocation-free batch entry point (this device is
       current): the device array's address, its host staging and event */
    e = qm::batch_scratch_address(hip_device, &c->noalloc_dev);
    if (e == hipSuccess) e = hipHostMalloc(&c->noalloc_host, qm::BATCH_SCRATCH_BYTES, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->noalloc_ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        if (c->noalloc_host) (void)hipHostFree(c->noalloc_host);
        delete c;
        return hip_fail(e, "set-up of the allocation-free batch path");
    }
    *out = c;
    return QM_OK;
}

void qm_shutdown(qm_ctx* ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->server) { qm::server_stop(ctx->server); ctx->server = nullptr; }
    qm::runner_free(ctx);
    for (auto& kv : ctx->tables) (void)hipFree(kv.second.d_table);
    for (auto& kv : ctx->hyp_tables) (void)hipFree(kv.second.d_table);
    for (auto& kv : ctx->vg_tables) (void)hipFree(kv.second.d_table);
    if (ctx->noalloc_ev) {
        (void)hipEventSynchronize(ctx->noalloc_ev);
        (void)hipEventDestroy(ctx->noalloc_ev);
    }
    if (ctx->noalloc_host) (void)hipHostFree(ctx->noalloc_host);
    delete ctx;
}

static qm_status single(qm_ctx* ctx, uint32_t kind, const void* in, void* out, uint64_t n, int dtype, int mode,
                        double nu, void* stream)
{
    if (!ctx) return fail(QM_E_INVAL, "context is NULL");
    qm_request r{};
    r.kind = kind;
    r.dtype = (uint32_t)dtype;
    r.mode = (uint32_t)mode;
    r.nu = nu;
    r.d_in = in;
    r.d_out = out;
    r.n = n;
    if (dtype != QM_F32 && dtype != QM_F64) return fail(QM_E_INVAL, "unknown dtype %d", dtype);
    if (!mode_known((uint32_t)mode)) return fail(QM_E_INVAL, "unknown mode %d", mode);
    qm_status st = qm::check_request(r, nullptr, true);
    if (st != QM_OK) return st;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return qm::run_single(ctx, r, (hipStream_t)stream);
}

qm_status qm_normal_quantile(qm_ctx* ctx, const void* d_u, void* d_w, uint64_t n, int dtype, int mode, void* s)
{
    return single(ctx, QM_NORMAL_QUANTILE, d_u, d_w, n, dtype, mode, 0.0, s);
}

qm_status qm_recycle_student_t(qm_ctx* ctx, const void* d_z, void* d_t, uint64_t n, int dtype, int mode,
                               double nu, void* s)
{
    return single(ctx, QM_STUDENT_T, d_z, d_t, n, dtype, mode, nu, s);
}

qm_status qm_recycle_exp_to_normal(qm_ctx* ctx, const void* d_x, void* d_z, uint64_t n, int dtype, int mode,
                                   void* s)
{
    return single(ctx, QM_EXP_TO_NORMAL, d_x, d_z, n, dtype, mode, 0.0, s);
}

qm_status qm_recycle_exp_to_hyperbolic(qm_ctx* ctx, const void* d_v, void* d_x, uint64_t n, int dtype, int mode,
                                       double alpha, double beta, double delta, double mu, void* s)
{
    if (!ctx) return fail(QM_E_INVAL, "context is NULL");
    if (dtype != QM_F32 && dtype != QM_F64) return fail(QM_E_INVAL, "unknown dtype %d", dtype);
    if (!mode_known((uint32_t)mode)) return fail(QM_E_INVAL, "unknown mode %d", mode);
    qm_request r{};
    r.kind = QM_EXP_TO_HYPERBOLIC;
    r.dtype = (uint32_t)dtype;
    r.mode = (uint32_t)mode;
    r.d_in = d_v;
    r.d_out = d_x;
    r.n = n;
    r.alpha = alpha;
    r.beta = beta;
    r.delta = delta;
    r.mu = mu;
    qm_status st = qm::check_request(r, nullptr, true);
    if (st != QM_OK) return st;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    /* the table is built (and cached) even for n = 0, so that a call can
       prepare it ahead of time */
    const DeviceHypTable* t = nullptr;
    st = qm::get_hyp_table(ctx, alpha, beta, delta, &t);
    if (st != QM_OK) return st;
    return qm::run_single(ctx, r, (hipStream_t)s);
}

qm_status qm_recycle_exp_to_vg(qm_ctx* ctx, const void* d_v, void* d_x, uint64_t n, int dtype, int mode, double lambda,
                               double alpha, double beta, double mu, void* s)
{
    if (!ctx) return fail(QM_E_INVAL, "context is NULL");
    if (dtype != QM_F32 && dtype != QM_F64) return fail(QM_E_INVAL, "unknown dtype %d", dtype);
    if (!mode_known((uint32_t)mode)) return fail(QM_E_INVAL, "unknown mode %d", mode);
    qm_request r{};
    r.kind = QM_EXP_TO_VG;
    r.dtype = (uint32_t)dtype;
    r.mode = (uint32_t)mode;
    r.nu = lambda;
    r.d_in = d_v;
    r.d_out = d_x;
    r.n = n;
    r.alpha = alpha;
    r.beta = beta;
    r.mu = mu;
    qm_status st = qm::check_request(r, nullptr, true);
    if (st != QM_OK) return st;
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    /* the table is built (and cached) even for n = 0 */
    const DeviceHypTable* t = nullptr;
    st = qm::get_vg_table(ctx, lambda, alpha, beta, &t);
    if (st != QM_OK) return st;
    return qm::run_single(ctx, r, (hipStream_t)s);
}

qm_status qm_vg_masses(qm_ctx* ctx, double lambda, double alpha, double beta, double* log_p_plus, double* log_p_minus)
{
    if (!ctx) return fail(QM_E_INVAL, "context is NULL");
    if (!vg_params_ok(lambda, alpha, beta))
        return fail(QM_E_INVAL, "need lambda in [1, 8] and |beta| < alpha, all finite (got %g, %g, %g)",
                    lambda, alpha, beta);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const DeviceHypTable* t = nullptr;
    qm_status st = qm::get_vg_table(ctx, lambda, alpha, beta, &t);
    if (st != QM_OK) return st;
    if (log_p_plus) *log_p_plus = t->hdr.log_p_plus;
    if (log_p_minus) *log_p_minus = t->hdr.log_p_minus;
    return QM_OK;
}

qm_status qm_hyperbolic_masses(qm_ctx* ctx, double alpha, double beta, double delta, double* log_p_plus,
                               double* log_p_minus)
{
    if (!ctx) return fail(QM_E_INVAL, "context is NULL");
    if (!hyp_params_ok(alpha, beta, delta))
        return fail(QM_E_INVAL, "need |beta| < alpha, delta > 0, all finite (got %g, %g, %g)", alpha, beta, delta);
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const DeviceHypTable* t = nullptr;
    qm_status st = qm::get_hyp_table(ctx, alpha, beta, delta, &t);
    if (st != QM_OK) return st;
    if (log_p_plus) *log_p_plus = t->hdr.log_p_plus;
    if (log_p_minus) *log_p_minus = t->hdr.log_p_minus;
    return QM_OK;
}

qm_status qm_generate(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                      int kind, int dtype, int mode, void* hs)
{
    if (!ctx) return fail(QM_E_INVAL, "context is NULL");
    if (seed > 0xFFFFFFFFull || stream > 0xFFFFFFFFull) return fail(QM_E_INVAL, "seed and stream must be < 2^32");
    if (dtype != QM_F32 && dtype != QM_F64) return fail(QM_E_INVAL, "unknown dtype %d", dtype);
    if (!mode_known((uint32_t)mode)) return fail(QM_E_INVAL, "unknown mode %d", mode);
    if (kind == QM_UNIFORM) {
        if (mode != QM_PLAIN) return fail(QM_E_DTYPE, "QM_UNIFORM takes mode QM_PLAIN");
    } else if (kind == QM_NORMAL_QUANTILE) {
        if (dtype == QM_F64 && mode == QM_F32_REFINE) return fail(QM_E_DTYPE, "QM_F32_REFINE needs dtype QM_F32");
        if (mode == QM_PAPER_T2) return fail(QM_E_INVAL, "QM_PAPER_T2 is a qm_normal_quantile mode only");
    } else {
        return fail(QM_E_INVAL, "qm_generate: kind must be QM_UNIFORM or QM_NORMAL_QUANTILE (got %d)", kind);
    }
    if (first > (1ull << 63) || n > (1ull << 63) - first) return fail(QM_E_INVAL, "first + n beyond 2^63");
    if (n == 0) return QM_OK;
    if (!d_out) return fail(QM_E_INVAL, "NULL output with n > 0");
    if ((uintptr_t)d_out % dtype_size(dtype)) return fail(QM_E_INVAL, "output must be aligned to the element size");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    e = qm::launch_generate(kind, dtype, mode, (uint32_t)seed, (uint32_t)stream, first, d_out, n, (hipStream_t)hs,
                            ctx->shape);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QM_OK;
}

/* The checks qm_generate makes of its stream arguments and output. */
static qm_status check_generate(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                                int dtype, int mode)
{
    if (!ctx) return fail(QM_E_INVAL, "context is NULL");
    if (seed > 0xFFFFFFFFull || stream > 0xFFFFFFFFull) return fail(QM_E_INVAL, "seed and stream must be < 2^32");
    if (dtype != QM_F32 && dtype != QM_F64) return fail(QM_E_INVAL, "unknown dtype %d", dtype);
    if (!mode_known((uint32_t)mode)) return fail(QM_E_INVAL, "unknown mode %d", mode);
    if (!(dtype == QM_F64 && mode == QM_PLAIN) && !(dtype == QM_F32 && mode == QM_F32_REFINE))
        return fail(QM_E_DTYPE, "F64 QM_PLAIN or F32 QM_F32_REFINE");
    if (first > (1ull << 63) || n > (1ull << 63) - first) return fail(QM_E_INVAL, "first + n beyond 2^63");
    if (n > 0 && !d_out) return fail(QM_E_INVAL, "NULL output with n > 0");
    if ((uintptr_t)d_out % dtype_size(dtype)) return fail(QM_E_INVAL, "output must be aligned to the element size");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return QM_OK;
}

qm_status qm_generate_student_t(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                                int dtype, int mode, double nu, void* hs)
{
    qm_status st = check_generate(ctx, seed, stream, first, d_out, n, dtype, mode);
    if (st != QM_OK) return st;
    if (std::isnan(nu) || !(nu >= qm::T_NU_MIN))
        return fail(QM_E_INVAL, "nu must be >= %g or +inf (got %g)", qm::T_NU_MIN, nu);
    const DeviceTable* t = nullptr;
    st = qm::get_table(ctx, nu, &t);
    if (st != QM_OK || n == 0) return st;
    hipError_t e = qm::launch_generate_student(dtype, mode, (uint32_t)seed, (uint32_t)stream, first, d_out, n,
                                               t->d_table, t->hdr, (hipStream_t)hs, ctx->shape);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QM_OK;
}

qm_status qm_generate_hyperbolic(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                                 int dtype, int mode, double alpha, double beta, double delta, double mu, void* hs)
{
    qm_status st = check_generate(ctx, seed, stream, first, d_out, n, dtype, mode);
    if (st != QM_OK) return st;
    if (!hyp_params_ok(alpha, beta, delta))
        return fail(QM_E_INVAL, "need |beta| < alpha, delta > 0, all finite (got %g, %g, %g)", alpha, beta, delta);
    if (!std::isfinite(mu)) return fail(QM_E_INVAL, "mu must be finite");
    const DeviceHypTable* t = nullptr;
    st = qm::get_hyp_table(ctx, alpha, beta, delta, &t);
    if (st != QM_OK || n == 0) return st;
    hipError_t e = qm::launch_generate_hyperbolic(dtype, mode, (uint32_t)seed, (uint32_t)stream, first, d_out, n,
                                                  t->d_table, t->hdr, t->ncoef, mu, (hipStream_t)hs, ctx->shape);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QM_OK;
}

qm_status qm_generate_vg(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                         int dtype, int mode, double lambda, double alpha, double beta, double mu, void* hs)
{
    qm_status st = check_generate(ctx, seed, stream, first, d_out, n, dtype, mode);
    if (st != QM_OK) return st;
    if (!vg_params_ok(lambda, alpha, beta))
        return fail(QM_E_INVAL, "need lambda in [1, 8] and |beta| < alpha, all finite (got %g, %g, %g)",
                    lambda, alpha, beta);
    if (!std::isfinite(mu)) return fail(QM_E_INVAL, "mu must be finite");
    const DeviceHypTable* t = nullptr;
    st = qm::get_vg_table(ctx, lambda, alpha, beta, &t);
    if (st != QM_OK || n == 0) return st;
    /* the same base and table format as the hyperbolic map */
    hipError_t e = qm::launch_generate_hyperbolic(dtype, mode, (uint32_t)seed, (uint32_t)stream, first, d_out, n,
                                                  t->d_table, t->hdr, t->ncoef, mu, (hipStream_t)hs, ctx->shape);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return QM_OK;
}

const char* qm_status_string(qm_status s)
{
    switch (s) {
    case QM_OK: return "QM_OK";
    case QM_PENDING: return "QM_PENDING";
    case QM_E_INVAL: return "QM_E_INVAL";
    case QM_E_DTYPE: return "QM_E_DTYPE";
    case QM_E_NOMEM: return "QM_E_NOMEM";
    case QM_E_HIP: return "QM_E_HIP";
    case QM_E_CLOSED: return "QM_E_CLOSED";
    case QM_E_TICKET: return "QM_E_TICKET";
    default: return "QM_UNKNOWN_STATUS";
    }
}

const char* qm_last_error(void) { return g_last_error.c_str(); }

}  /* extern "C" */

/* Error helpers for the other translation units. */
namespace qm {
qm_status set_error(qm_status s, const char* msg) { return fail(s, "%s", msg); }
}
