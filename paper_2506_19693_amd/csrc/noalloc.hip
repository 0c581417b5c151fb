// Allocation-free rescale for callers that cannot allocate device memory
// (work recorded under stream capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The rescale's scratch (the two last limbs after their inverse NTT and the
// lifted limbs, 2 count (1 + l) N words) lives in `scratch`, a file-scope
// device array of RBK_NOALLOC_SCRATCH_BYTES.  Each GPU the library runs on
// holds its own copy at its own address until the process ends.  In host
// code the array's name is only a stand-in, so its device address is looked
// up once per device with hipGetSymbolAddress (with that device current, when
// the first context on it is created) and only that address is handed to the
// kernels.  Nothing the rescale reads from the scratch needs to start at
// zero: every word is written before it is read within one call.  Calls that
// overlap in time on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/rbk.h"
#include "rbk_ctx.hpp"

namespace {

constexpr size_t SCRATCH_WORDS = RBK_NOALLOC_SCRATCH_BYTES / sizeof(u64);
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) u64 scratch[SCRATCH_WORDS];

u64 *scratch_dev[MAX_DEVICES];  // per device: the address of that device's copy
std::mutex scratch_mu;

}  // namespace

int noalloc_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return rbk_set_error(RBK_EUNSUPPORTED, "device index above 63");
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_dev[device]) return RBK_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return rbk_set_error(RBK_EDEVICE, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    scratch_dev[device] = (u64 *)p;
    return RBK_OK;
}

extern "C" int rbk_rescale_batch_noalloc(rbk_ctx *c, const uint64_t *ct, uint64_t *out, int level, int count)
{
    int rc = rescale_check(c, ct, out, level, count);
    if (rc) return rc;
    if (c->timing) return rbk_set_error(RBK_ESTATE, "per-kernel timers are on (they create events)");
    if ((size_t)count > SCRATCH_WORDS / c->N || rescale_ws_words(c, level, count) > SCRATCH_WORDS)
        return rbk_set_error(RBK_EINVAL, "rescale needs 2 x count x (1 + level) x N words of scratch, "
                                         "above RBK_NOALLOC_SCRATCH_BYTES");
    u64 *ws = (c->device >= 0 && c->device < MAX_DEVICES) ? scratch_dev[c->device] : nullptr;
    if (!ws) return rbk_set_error(RBK_ESTATE, "scratch address of this device not set up");
    return rescale_run(c, ct, out, level, count, ws);
}
