// abm_solve_noalloc: the plain per-step solve of one trajectory (as
// abm_solve) for callers that cannot allocate device memory.  Everything the
// kernels need beyond the caller's problem and output lives in `scratch`, a
// file-scope device array each GPU holds until the process ends:
//
//   [0, 256)            status word (kStatus* bits)
//   [256, 1280)         step flags of the cooperative form (256 x uint32)
//   [1280, 1280 + 32K)  partial slots of the cooperative form (2 x 256 x 8 doubles)
//   then per distinct order: Gamma(alpha+1), Gamma(alpha+2) (256 B), then
//   b, a, c, each N + kWeightPad doubles (256-byte aligned).
//
// The host never uses the array's name as an address: the device address of
// each GPU's copy comes from hipGetSymbolAddress, taken once per device with
// that device current, and that pointer is what the kernels receive.  Nothing
// here allocates; the launches are the weight kernel, the fill kernel and the
// plain kernel of abm_solve, with the same launch shape, so the results are
// bitwise those of abm_solve.
#include <hip/hip_runtime.h>

#include <mutex>

#include "abm.h"
#include "abm_kernels.h"
#include "abm_runtime.h"

namespace abm {

namespace {

constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr size_t kStatusOff = 0;
constexpr size_t kFlagsOff = 256;
constexpr size_t kPartOff = 1280;
constexpr size_t kTablesOff = kPartOff + 8 * 256 * 8 * sizeof(double);   // plain_part_doubles(256)
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// This device's copy of scratch (the current device).
abm_status scratch_of(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(ABM_EINVAL, "device %d", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_ptr[dev];
    return ABM_OK;
}

// Workspace bytes one problem takes (status, flags, partials, its tables).
size_t noalloc_bytes_needed(const abm_problem& p)
{
    double seen[4];
    int ntab = 0;
    for (int i = 0; i < p.d; ++i) {
        const double al = order_of(p, i);
        bool dup = false;
        for (int t = 0; t < ntab; ++t) dup |= seen[t] == al;
        if (!dup) seen[ntab++] = al;
    }
    const size_t table = 256 + 3 * align256((size_t)(p.N + kWeightPad) * sizeof(double));
    return kTablesOff + (size_t)ntab * table;
}

}  // namespace

}  // namespace abm

using namespace abm;

extern "C" abm_status abm_solve_noalloc(const abm_problem* prob, double* y_out, void* hip_stream)
{
    if (!prob || !y_out) return fail(ABM_EINVAL, "NULL argument");
    abm_status s = validate(*prob, 0);
    if (s != ABM_OK) return s;
    if (prob->far_prec == ABM_FAR_DD)
        return fail(ABM_EINVAL, "double-double (ABM_FAR_DD) runs on abm_solve only");
    const size_t need = noalloc_bytes_needed(*prob);
    if (need > kScratchBytes)
        return fail(ABM_EINVAL,
                    "N=%lld needs %zu bytes of the no-allocation workspace, which holds %zu",
                    (long long)prob->N, need, kScratchBytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    int n_cu = 0;
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    PlainShape sh{};
    if ((s = plain_shape(*prob, n_cu, &sh)) != ABM_OK) return s;
    if ((size_t)plain_part_doubles(sh.G) * sizeof(double) > kTablesOff - kPartOff)
        return fail(ABM_EINVAL, "%d workgroups' partial slots exceed the workspace layout", sh.G);
    unsigned char* base = nullptr;
    if ((s = scratch_of(dev, &base)) != ABM_OK) return s;
    const hipStream_t st = (hipStream_t)hip_stream;

    // weight tables, one per distinct order (components of equal order share)
    PlainTables T{};
    double orders[4];
    unsigned char* tab[4];
    int ntab = 0;
    const int64_t wn = prob->N + kWeightPad;
    const size_t arr = align256((size_t)wn * sizeof(double));
    for (int i = 0; i < 4; ++i) {
        const double al = order_of(*prob, i < prob->d ? i : 0);
        int t = 0;
        while (t < ntab && orders[t] != al) ++t;
        if (t == ntab) {
            orders[ntab] = al;
            tab[ntab] = base + kTablesOff + (size_t)ntab * (256 + 3 * arr);
            double* gam = reinterpret_cast<double*>(tab[ntab]);
            double* b = reinterpret_cast<double*>(tab[ntab] + 256);
            double* a = reinterpret_cast<double*>(tab[ntab] + 256 + arr);
            double* c = reinterpret_cast<double*>(tab[ntab] + 256 + 2 * arr);
            if ((e = launch_weights(al, wn, gam, b, a, c, st)) != hipSuccess)
                return hip_fail(e, "weight kernel");
            ++ntab;
        }
        T.gam[i] = reinterpret_cast<const double*>(tab[t]);
        T.b[i] = reinterpret_cast<const double*>(tab[t] + 256);
        T.a[i] = reinterpret_cast<const double*>(tab[t] + 256 + arr);
        T.c[i] = reinterpret_cast<const double*>(tab[t] + 256 + 2 * arr);
        T.alpha[i] = al;
    }
    uint32_t* status = reinterpret_cast<uint32_t*>(base + kStatusOff);
    if ((e = launch_fill_u32(status, 0, 1, st)) != hipSuccess) return hip_fail(e, "status reset");
    const PlainArgs A =
        plain_args(*prob, T, sh, reinterpret_cast<double*>(base + kPartOff),
                   reinterpret_cast<uint32_t*>(base + kFlagsOff), status, y_out);
    if ((e = plain_enqueue(A, sh, chain_kind(prob->rhs, orders_differ(*prob)), st)) != hipSuccess)
        return hip_fail(e, "plain kernel launch");
    return ABM_OK;
}
