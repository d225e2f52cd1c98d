// libabm runtime: contexts, plans, argument checking and the C ABI entry
// points declared in include/abm.h.  Every arithmetic step of the method runs
// in the kernels (K0 weights, K1 plain path, far-field and chain kernels of
// the blocked path); this file only validates, allocates and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "abm.h"
#include "abm_kernels.h"
#include "abm_runtime.h"

namespace abm {

static thread_local std::string g_last_error;

abm_status fail(abm_status code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

abm_status hip_fail(hipError_t e, const char* what)
{
    return fail(e == hipErrorOutOfMemory ? ABM_ENOMEM : ABM_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

int rhs_dim(int rhs)
{
    switch (rhs) {
    case ABM_RHS_LINEAR: return 1;
    case ABM_RHS_DUFFING: return 2;
    case ABM_RHS_LORENZ: return 3;
    case ABM_RHS_POLY: return 1;
    case ABM_RHS_LCR: return 2;
    case ABM_RHS_DIAG: return 2;
    default: return -1;
    }
}

double order_of(const abm_problem& p, int comp)
{
    return p.alphas[0] > 0.0 ? p.alphas[comp] : p.alpha;
}

bool orders_differ(const abm_problem& p)
{
    for (int i = 1; i < p.d; ++i)
        if (order_of(p, i) != order_of(p, 0)) return true;
    return false;
}

int deriv_mask(const abm_problem& p)
{
    int m = 0;
    for (int i = 0; i < p.d; ++i)
        if (order_of(p, i) > 1.0) m |= 1 << i;
    return m;
}

bool same_orders(const abm_problem& a, const abm_problem& b)
{
    if (a.d != b.d) return false;
    for (int i = 0; i < a.d; ++i)
        if (order_of(a, i) != order_of(b, i)) return false;
    return true;
}

int64_t n_out(int64_t N, int64_t stride)
{
    if (stride == 0) return 1;
    return N / stride + 1 + (N % stride ? 1 : 0);
}

abm_status validate(const abm_problem& p, int idx)
{
    const int d = rhs_dim(p.rhs);
    if (d < 0) return fail(ABM_EINVAL, "problem %d: unknown rhs %d", idx, p.rhs);
    if (p.d != d) return fail(ABM_EINVAL, "problem %d: d=%d but rhs %d has dimension %d", idx, p.d, p.rhs, d);
    for (int i = 0; i < d; ++i) {
        const double al = order_of(p, i);
        if (!(al > 0.0 && al <= 2.0))
            return fail(ABM_EINVAL, "problem %d: order %g of component %d outside (0, 2]", idx, al, i);
        if (al > 1.0 && !std::isfinite(p.x1[i]))
            return fail(ABM_EINVAL, "problem %d: x1 not finite", idx);
    }
    if (!(p.h > 0.0) || !std::isfinite(p.h))
        return fail(ABM_EINVAL, "problem %d: h=%g must be positive and finite", idx, p.h);
    if (p.N < 1 || p.N > kMaxSteps)
        return fail(ABM_EINVAL, "problem %d: N=%lld outside [1, %lld]", idx, (long long)p.N,
                    (long long)kMaxSteps);
    if (p.out_stride < 0) return fail(ABM_EINVAL, "problem %d: out_stride < 0", idx);
    if (p.far_prec < ABM_FAR_FP64 || p.far_prec > ABM_FAR_I8)
        return fail(ABM_EINVAL, "problem %d: unknown far_prec %d", idx, p.far_prec);
    for (int i = 0; i < d; ++i)
        if (!std::isfinite(p.x0[i])) return fail(ABM_EINVAL, "problem %d: x0 not finite", idx);
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(p.p[i])) return fail(ABM_EINVAL, "problem %d: p not finite", idx);
    return ABM_OK;
}

// Shape fields a plan fixes; x0, p and h may change between solves.
static bool same_shape(const abm_problem& a, const abm_problem& b)
{
    return a.rhs == b.rhs && a.d == b.d && same_orders(a, b) && a.N == b.N &&
           a.far_prec == b.far_prec && a.out_stride == b.out_stride;
}

int env_int(const char* name, int dflt)
{
    const char* v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}

abm_status dev_alloc(void** p, size_t bytes, const char* what)
{
    *p = nullptr;
    if (bytes == 0) return ABM_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, what);
    }
    return ABM_OK;
}

void dev_free(void* p)
{
    if (p) (void)hipFree(p);
}

static void free_tables(abm_plan_s* pl)
{
    for (auto& t : pl->tables) {
        dev_free(t.gam);
        dev_free(t.b);
        dev_free(t.a);
        dev_free(t.c);
        free_reduced(t);
    }
    pl->tables.clear();
}

}  // namespace abm

using namespace abm;

extern "C" {

const char* abm_strerror(abm_status s)
{
    switch (s) {
    case ABM_OK: return "ok";
    case ABM_EINVAL: return "invalid argument";
    case ABM_ENOMEM: return "out of memory";
    case ABM_EDEVICE: return "device failure";
    case ABM_EAGAIN: return "not finished";
    case ABM_ENOENT: return "unknown ticket";
    case ABM_ECANCELED: return "cancelled";
    default: return "unknown status";
    }
}

const char* abm_last_error(void) { return g_last_error.c_str(); }

abm_status abm_ctx_create(int device, void* hip_stream, size_t arena_bytes, abm_ctx** out)
{
    if (!out) return fail(ABM_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(ABM_EINVAL, "device %d of %d", device, n);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    abm_ctx* c = new abm_ctx();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->arena_bytes = arena_bytes ? arena_bytes : ((size_t)1 << 30);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipGetDeviceProperties");
    }
    c->n_cu = prop.multiProcessorCount;
    // the serving state exists from the start (its thread and device memory
    // only from the first submit), so concurrent first submits and polls
    // never race to create it
    abm_status s = serve_create(c);
    if (s != ABM_OK) {
        delete c;
        return s;
    }
    *out = c;
    return ABM_OK;
}

void abm_ctx_destroy(abm_ctx* ctx)
{
    if (!ctx) return;
    serve_shutdown(ctx);
    delete ctx;
}

abm_status abm_plan(abm_ctx* ctx, const abm_problem* probs, int32_t B, abm_plan_t** out)
{
    return abm_plan_tuned(ctx, probs, B, nullptr, out);
}

abm_status abm_plan_tuned(abm_ctx* ctx, const abm_problem* probs, int32_t B,
                          const abm_tuning* tune, abm_plan_t** out)
{
    if (!ctx || !probs || !out) return fail(ABM_EINVAL, "NULL argument");
    *out = nullptr;
    if (B < 1) return fail(ABM_EINVAL, "B=%d must be >= 1", B);
    for (int i = 0; i < B; ++i) {
        abm_status s = validate(probs[i], i);
        if (s != ABM_OK) return s;
    }
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    bool dd = false;
    for (int i = 0; i < B; ++i) dd |= probs[i].far_prec == ABM_FAR_DD;
    if (dd && B != 1)
        return fail(ABM_EINVAL, "double-double (ABM_FAR_DD) runs one trajectory per plan, on abm_solve");
    abm_plan_s* pl = new abm_plan_s();
    pl->ctx = ctx;
    pl->B = B;
    pl->dd = dd;
    pl->shape.assign(probs, probs + B);
    if (tune) pl->tune = *tune;
    abm_status st = ABM_OK;

    // one weight table per distinct order, long enough for its longest user
    pl->table_of.assign((size_t)B * 4, 0);
    for (int i = 0; i < B; ++i) {
        for (int c = 0; c < probs[i].d; ++c) {
            const double al = order_of(probs[i], c);
            int found = -1;
            for (size_t j = 0; j < pl->tables.size(); ++j)
                if (pl->tables[j].alpha == al) found = (int)j;
            if (found < 0) {
                WeightTable t{};
                t.alpha = al;
                pl->tables.push_back(t);
                found = (int)pl->tables.size() - 1;
            }
            pl->tables[found].n = std::max<int64_t>(pl->tables[found].n, probs[i].N);
            pl->table_of[(size_t)i * 4 + c] = found;
        }
        for (int c = probs[i].d; c < 4; ++c) pl->table_of[(size_t)i * 4 + c] = pl->table_of[(size_t)i * 4];
    }
    for (auto& t : pl->tables) {
        // padded so that block kernels may read a full tile past N; a
        // double-double table holds (hi, lo) pairs
        const int64_t n = t.n + kWeightPad;
        const size_t w = dd ? 2 : 1;
        if ((st = dev_alloc((void**)&t.gam, 2 * w * sizeof(double), "weights")) ||
            (st = dev_alloc((void**)&t.b, w * n * sizeof(double), "weights")) ||
            (st = dev_alloc((void**)&t.a, w * n * sizeof(double), "weights")) ||
            (st = dev_alloc((void**)&t.c, w * n * sizeof(double), "weights")))
            break;
        e = dd ? launch_weights_dd(t.alpha, n, t.gam, t.b, t.a, t.c, ctx->stream)
               : launch_weights(t.alpha, n, t.gam, t.b, t.a, t.c, ctx->stream);
        if (e != hipSuccess) {
            st = hip_fail(e, "weight kernel");
            break;
        }
    }
    if (st == ABM_OK) st = dev_alloc((void**)&pl->status, sizeof(uint32_t), "status");
    if (st == ABM_OK) {
        e = launch_fill_u32(pl->status, 0, 1, ctx->stream);
        if (e != hipSuccess) st = hip_fail(e, "fill");
    }
    if (st == ABM_OK && dd) {
        // double-double: the plain path only, and it must fit
        st = plain_setup_dd(pl);
    } else if (st == ABM_OK && B == 1) {
        // the plain path is optional: a history too long for it leaves plain_G = 0
        const abm_status ps = plain_setup(pl);
        if (ps == ABM_ENOMEM || ps == ABM_EDEVICE) st = ps;
        if (ps != ABM_OK) pl->plain_error = abm_last_error();
    }
    if (st == ABM_OK && !dd) st = batch_setup(pl);
    if (st != ABM_OK) {
        abm_plan_destroy(pl);
        return st;
    }
    *out = pl;
    return ABM_OK;
}

void abm_plan_destroy(abm_plan_t* pl)
{
    if (!pl) return;
    (void)hipSetDevice(pl->ctx->device);
    (void)hipStreamSynchronize(pl->ctx->stream);
    free_tables(pl);
    dev_free(pl->part);
    dev_free(pl->flags);
    dev_free(pl->status);
    batch_teardown(pl);
    delete pl;
}

abm_status abm_plan_check(abm_plan_t* pl)
{
    if (!pl) return fail(ABM_EINVAL, "plan is NULL");
    hipError_t e = hipStreamSynchronize(pl->ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    uint32_t bits = 0;
    e = hipMemcpy(&bits, pl->status, sizeof bits, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "status read");
    if (bits) {
        (void)launch_fill_u32(pl->status, 0, 1, pl->ctx->stream);
        (void)hipStreamSynchronize(pl->ctx->stream);
        return fail(ABM_EDEVICE, "device status 0x%x (%s%s)", bits,
                    (bits & 1u) ? "wait timed out " : "", (bits & 2u) ? "non-finite state" : "");
    }
    return ABM_OK;
}

abm_status abm_plan_weights(abm_plan_t* pl, int32_t idx, int64_t n, double* b, double* a,
                            double* c)
{
    if (!pl) return fail(ABM_EINVAL, "plan is NULL");
    if (idx < 0 || idx >= pl->B) return fail(ABM_EINVAL, "idx %d outside [0, %d)", idx, pl->B);
    const WeightTable& t = pl->tables[pl->table_of[(size_t)idx * 4]];
    if (n < 0 || n > t.n + kWeightPad)
        return fail(ABM_EINVAL, "n=%lld outside [0, %lld]", (long long)n, (long long)(t.n + kWeightPad));
    const size_t bytes = (pl->dd ? 2 : 1) * n * sizeof(double);
    hipError_t e = hipSetDevice(pl->ctx->device);
    if (e == hipSuccess) e = hipStreamSynchronize(pl->ctx->stream);
    if (e == hipSuccess && b) e = hipMemcpy(b, t.b, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && a) e = hipMemcpy(a, t.a, bytes, hipMemcpyDeviceToHost);
    if (e == hipSuccess && c) e = hipMemcpy(c, t.c, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "weight copy");
    return ABM_OK;
}

abm_status abm_solve(abm_plan_t* pl, const abm_problem* prob, double* y_out)
{
    if (!pl || !prob || !y_out) return fail(ABM_EINVAL, "NULL argument");
    if (pl->B != 1) return fail(ABM_EINVAL, "abm_solve needs a plan made for one problem (B=%d)", pl->B);
    if (pl->plain_G <= 0) return fail(ABM_EINVAL, "plain path unavailable: %s", pl->plain_error.c_str());
    abm_status s = validate(*prob, 0);
    if (s != ABM_OK) return s;
    if (!same_shape(*prob, pl->shape[0]))
        return fail(ABM_EINVAL, "problem does not match the plan (rhs, d, orders, N, far_prec, out_stride)");
    hipError_t e = hipSetDevice(pl->ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    PlainTables T{};
    for (int i = 0; i < 4; ++i) {
        const WeightTable& t = pl->tables[pl->table_of[i]];
        T.b[i] = t.b;
        T.a[i] = t.a;
        T.c[i] = t.c;
        T.gam[i] = t.gam;
        T.alpha[i] = t.alpha;
    }
    const PlainShape sh{pl->plain_single, pl->plain_G, pl->plain_nloc};
    const PlainArgs A = plain_args(*prob, T, sh, pl->part, pl->flags, pl->status, y_out);
    const int kind = chain_kind(prob->rhs, orders_differ(*prob));
    if (pl->dd) {
        if (!sh.single && (e = launch_fill_u32(A.flags, 0, sh.G, pl->ctx->stream)) != hipSuccess)
            return hip_fail(e, "flag reset");
        e = launch_plain_dd(A, sh.single, kind, pl->ctx->stream);
    } else {
        e = plain_enqueue(A, sh, kind, pl->ctx->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "plain kernel launch");
    return ABM_OK;
}

}  // extern "C"

namespace abm {

abm_status plain_shape(const abm_problem& p, int n_cu, PlainShape* out)
{
    const int ch = plain_chunk();
    const int64_t nchunks = std::max<int64_t>(1, (p.N + ch - 1) / ch);   // indices 0..N-1
    const int nloc_max = plain_max_local_chunks(p.d);
    // co-residency bound: one workgroup per CU is always possible for this kernel
    const int gcap = std::min(n_cu, 256);
    const int gmin = (int)((nchunks + nloc_max - 1) / nloc_max);
    if (gmin > gcap)
        return fail(ABM_EINVAL, "N=%lld too long for the plain path (history does not fit the LDS of %d workgroups)",
                    (long long)p.N, gcap);
    // a history that fits one CU runs in one workgroup with no grid
    // synchronisation (unless a workgroup count is forced)
    const int tables = orders_differ(p) ? p.d : 1;
    int G = env_int("ABM_PLAIN_G", 0);
    if (G <= 0 && plain_single_fits(p.N, p.d, tables)) {
        *out = PlainShape{true, 1, 0};
        return ABM_OK;
    }
    // otherwise the fewest workgroups whose local chunks all fit the
    // kernel's register prefetch (no weight load on a step's dependent path)
    const int pref = plain_prefetch_chunks(tables);
    if (G <= 0) G = (int)((nchunks + pref - 1) / pref);
    G = std::max(G, gmin);
    G = std::min(G, gcap);
    *out = PlainShape{false, G, (int)((nchunks + G - 1) / G)};
    return ABM_OK;
}

PlainArgs plain_args(const abm_problem& prob, const PlainTables& T, const PlainShape& sh,
                     double* part, uint32_t* flags, uint32_t* status, double* y_out)
{
    PlainArgs A{};
    for (int i = 0; i < 4; ++i) {
        A.b[i] = T.b[i];
        A.a[i] = T.a[i];
        A.c[i] = T.c[i];
        A.gam[i] = T.gam[i];
        A.alpha[i] = T.alpha[i];
        A.x0[i] = prob.x0[i];
        A.x1[i] = prob.x1[i];
    }
    A.h = prob.h;
    for (int i = 0; i < 8; ++i) A.p[i] = prob.p[i];
    A.N = prob.N;
    A.G = sh.G;
    A.nloc = sh.nloc;
    A.part = part;
    A.flags = flags;
    A.y_out = y_out;
    A.out_stride = prob.out_stride;
    A.status = status;
    // test hooks for the device-side waits' failure path: a smaller bound
    // and an offset that no flag reaches (every wait then gives up)
    const int spin = env_int("ABM_SPIN_LIMIT", 0);
    A.spin_limit = spin > 0 ? (uint32_t)spin : kSpinLimit;
    A.wait_bias = (uint32_t)std::max(0, env_int("ABM_WAIT_BIAS", 0));
    return A;
}

hipError_t plain_enqueue(const PlainArgs& A, const PlainShape& sh, int kind, hipStream_t st)
{
    if (sh.single) return launch_plain_single(A, kind, st);
    hipError_t e = launch_fill_u32(A.flags, 0, sh.G, st);
    if (e != hipSuccess) return e;
    return launch_plain(A, kind, st);
}

abm_status plain_setup_dd(abm_plan_s* pl)
{
    const abm_problem& p = pl->shape[0];
    const int tables = orders_differ(p) ? p.d : 1;
    int G = env_int("ABM_PLAIN_G", 0);
    if (G <= 0 && plain_dd_single_fits(p.N, p.d, tables)) {
        pl->plain_single = true;
        pl->plain_G = 1;
        pl->plain_nloc = 0;
        return ABM_OK;
    }
    const int ch = plain_chunk();
    const int64_t nchunks = std::max<int64_t>(1, (p.N + ch - 1) / ch);
    const int nloc_max = plain_dd_max_local_chunks(p.d);
    const int gcap = std::min(pl->ctx->n_cu, 256);
    const int gmin = (int)((nchunks + nloc_max - 1) / nloc_max);
    if (gmin > gcap)
        return fail(ABM_EINVAL, "N=%lld too long for the double-double plain path (history does not "
                    "fit the LDS of %d workgroups)", (long long)p.N, gcap);
    // four local chunks per workgroup: the most whose weights the kernel
    // prefetches into registers (measured on the 200000-step oscillator:
    // 6.3 us per step at 4 chunks, 7.1-7.3 at 5 to 8 with the weights loaded
    // in the step); short histories spread over at least 32 workgroups while
    // there are chunks for them (8192 steps: 2.39 us per step at 32, 2.55 at 8)
    if (G <= 0) G = (int)std::max<int64_t>((nchunks + 3) / 4, std::min<int64_t>(nchunks, 32));
    G = std::min(std::max(G, gmin), gcap);
    pl->plain_single = false;
    pl->plain_G = G;
    pl->plain_nloc = (int)((nchunks + G - 1) / G);
    abm_status st = dev_alloc((void**)&pl->part, plain_dd_part_doubles(G) * sizeof(double),
                              "plain partials");
    if (st == ABM_OK) st = dev_alloc((void**)&pl->flags, G * sizeof(uint32_t), "plain flags");
    return st;
}

abm_status plain_setup(abm_plan_s* pl)
{
    PlainShape sh{};
    abm_status st = plain_shape(pl->shape[0], pl->ctx->n_cu, &sh);
    if (st != ABM_OK) return st;
    pl->plain_single = sh.single;
    pl->plain_G = sh.G;
    pl->plain_nloc = sh.nloc;
    if (sh.single) return ABM_OK;
    st = dev_alloc((void**)&pl->part, plain_part_doubles(sh.G) * sizeof(double), "plain partials");
    if (st == ABM_OK) st = dev_alloc((void**)&pl->flags, sh.G * sizeof(uint32_t), "plain flags");
    return st;
}

}  // namespace abm
