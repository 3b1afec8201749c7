// kd_noalloc.hip -- kd_knn_noalloc: the plain kNN query with no device
// allocation.  Its scratch (query records, sort buffers, work counters,
// hand-off rows) lives in one fixed array of this library's code object
// instead of the per-stream buffer the other query calls allocate on demand,
// so the call suits code that must not allocate (stream capture, tight
// serving loops).  Results and kernels are those of kd_knn.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "kd_internal.h"

// The fixed scratch.  Each device the library runs on holds its own copy
// from module load until the process ends.  Host code never passes this
// name to a kernel: its device address comes from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[KD_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_noalloc_mu;
std::map<int, void*> g_noalloc_ptr;  // device ordinal -> that device's copy of `scratch`

// Device address of the current device's copy of `scratch`, looked up once per
// device (with that device current) and cached.
kd_status noalloc_scratch(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_ptr.find(device);
    if (it != g_noalloc_ptr.end()) {
        *out = it->second;
        return KD_OK;
    }
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return kd::hip_error(e, "kd_knn_noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return kd::set_error(KD_EHIP, "kd_knn_noalloc: hipGetSymbolAddress(scratch) returned NULL");
    g_noalloc_ptr.emplace(device, p);
    *out = p;
    return KD_OK;
}

}  // namespace

extern "C" kd_status kd_knn_noalloc(kd_tree t, const float* queries, int64_t Q, int k, float maxRadius,
                                    int32_t* out_idx, float* out_d2, kd_stream stream) {
    kd_status s = kd::check_query_args_public(t, queries, Q, k, maxRadius, out_idx, "kd_knn_noalloc");
    if (s != KD_OK) return s;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return kd::hip_error(e, "kd_knn_noalloc: hipGetDevice");
    if (dev != t->device)
        return kd::set_error(KD_EINVAL, "kd_knn_noalloc: the tree lives on another device than the current one");
    void* ws = nullptr;
    s = noalloc_scratch(dev, &ws);
    if (s != KD_OK) return s;
    const kd::FixedScratch fixed{ws, size_t(KD_NOALLOC_SCRATCH_BYTES)};
    return kd::knn_entry(t, queries, Q, k, maxRadius, out_idx, out_d2, nullptr, nullptr, stream, "kd_knn_noalloc",
                         &fixed);
}
