// Tree forces without any device allocation: tpm_compute_forces_noalloc.
//
// tpm_compute_forces keeps its per-call working memory (the active set's
// marks, slot lists and compaction counts, and the walk results in slot
// order) in buffers of the context, which it (re)allocates when a tree grows.
// Callers that cannot allocate (code under stream capture, tight serving
// loops, harnesses that forbid allocation) use this variant instead: the
// same kernels, with that working memory in one file-scope device array of
// fixed size.  Each GPU holds its own copy of the array for the lifetime of
// the process; its device address is looked up once per device when a
// context is created there (tpm_create -> noalloc_attach) and kept per
// device.  Every call on a device shares that device's array: calls that
// overlap on one GPU (several streams or threads) race.
#include <mutex>

#include "tpm_internal.h"

namespace tpm {
namespace {

// Largest tree the array serves, and its layout (byte offsets, 256-aligned):
// marks, active slots, slot map, results [n][4] (acceleration and interaction
// count) and potentials [n] in FP64, compaction tile counts, and the
// unique-active counter.
constexpr int64_t kMaxN = int64_t(1) << 20;
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kOffMark = 0;
constexpr size_t kOffAct = kOffMark + align256(4 * kMaxN);
constexpr size_t kOffSlot = kOffAct + align256(4 * kMaxN);
constexpr size_t kOffRes = kOffSlot + align256(4 * kMaxN);
constexpr size_t kOffPot = kOffRes + align256(4 * 8 * kMaxN);
constexpr size_t kOffCounts = kOffPot + align256(8 * kMaxN);
constexpr size_t kOffNuniq = kOffCounts + align256(4 * kMaxN / 64 + 64);
constexpr size_t kScratchBytes = kOffNuniq + 256;  // 52 MiB + 17 KiB

// In host code this name is only a stand-in for the device symbol: kernels
// and copies receive the address kept in g_scratch[device] instead.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void *g_scratch[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};
bool g_looked_up[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the array (once per device; the device is
// current).  A failed lookup is remembered and reported by the entry point.
void noalloc_attach(int device) {
    if (device < 0 || device >= kMaxDevices)
        return;
    std::lock_guard<std::mutex> g(g_lock);
    if (g_looked_up[device])
        return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_looked_up[device] = true;
    g_status[device] = e;
    g_scratch[device] = e == hipSuccess ? p : nullptr;
    if (e != hipSuccess)
        (void)hipGetLastError();
}

int64_t noalloc_max_n() { return kMaxN; }

}  // namespace tpm

using namespace tpm;

extern "C" {

int64_t tpm_noalloc_max_n(void) { return kMaxN; }

int tpm_compute_forces_noalloc(tpm_ctx *c, int32_t opening, int64_t n_act,
                               const int32_t *idx, const double *anorm, void *acc, void *pot,
                               uint32_t *nint) {
    if (!c)
        return TPM_EINVAL;
    if (!c->built)
        return fail(c, TPM_ESTATE, "compute_forces_noalloc before build_tree");
    if (c->n > kMaxN)
        return fail(c, TPM_EINVAL,
                    "compute_forces_noalloc serves trees of at most 2^20 particles (this one has " +
                        std::to_string(c->n) + ")");
    if (opening != TPM_OPEN_BH && opening != TPM_OPEN_REL)
        return fail(c, TPM_EINVAL, "opening must be TPM_OPEN_BH or TPM_OPEN_REL");
    if (n_act < 0 || n_act > (int64_t(1) << 31) - 1)
        return fail(c, TPM_EINVAL, "n_act out of range");
    if (n_act > 0 && (!idx || !acc))
        return fail(c, TPM_EINVAL, "active_idx and acc must not be NULL");
    if (opening == TPM_OPEN_REL && n_act > 0 && !anorm)
        return fail(c, TPM_EINVAL, "the relative criterion needs a_old_norm");
    if (c->device < 0 || c->device >= kMaxDevices)
        return fail(c, TPM_EDEVICE, "device index beyond the scratch table");
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_lock);
        if (!g_looked_up[c->device])
            return fail(c, TPM_ESTATE, "scratch of this device was not looked up");
        if (g_status[c->device] != hipSuccess)
            return fail(c, TPM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                            hipGetErrorString(g_status[c->device]));
        base = g_scratch[c->device];
    }
    if (n_act == 0)
        return TPM_OK;
    TPM_HIP(c, hipSetDevice(c->device));
    unsigned char *s = (unsigned char *)base;
    Work w;
    w.mark = (uint32_t *)(s + kOffMark);
    w.epoch = 1;
    w.clear = true;  // the array keeps the marks of the last call of any context
    w.act = (uint32_t *)(s + kOffAct);
    w.slot = (uint32_t *)(s + kOffSlot);
    w.res = s + kOffRes;
    w.rpot = s + kOffPot;
    w.counts = (uint32_t *)(s + kOffCounts);
    w.nuniq = (uint32_t *)(s + kOffNuniq);
    return forces_into(c, opening, n_act, idx, anorm, acc, pot, nint, w, false);
}

}  // extern "C"
