// Set-up check of a device view list, the rows of the minibatch selection M_k
// (Sec. 2.1, Eq. (7)), against a plan. The projectors and pnp_step read such a
// list on the device and treat an index outside [0, n_views) as a zero row;
// checking it there would cost a device-to-host copy per call, so callers that
// want the check make this call once, when they build the list.
#include <climits>
#include <string>

#include <hip/hip_runtime.h>

#include "fbpnp.h"
#include "fbpnp_impl.h"

namespace {

// *first = the smallest position i < n whose index lies outside [0, n_views)
__global__ __launch_bounds__(256) void k_check_views(const int32_t* __restrict__ views, int n, int n_views,
                                                     int* __restrict__ first) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n && (unsigned)views[i] >= (unsigned)n_views) atomicMin(first, i);
}

}  // namespace

extern "C" fb_status fb_check_views(const fb_plan* p, const int32_t* views, int32_t n_sel, hipStream_t stream) {
    using namespace fbpnp;
    if (!p) return fail(FB_EINVAL, "fb_check_views: plan is NULL");
    if (!views) return fail(FB_EINVAL, "fb_check_views: views is NULL");
    if (n_sel < 1) return fail(FB_EINVAL, "fb_check_views: n_sel must be positive");
    if (n_sel > p->g.n_views)
        return fail(FB_ESUBSET, "fb_check_views: " + std::to_string(n_sel) + " views listed, the plan has " +
                                    std::to_string(p->g.n_views));
    int* d = nullptr;
    if (hipMalloc(&d, sizeof(int)) != hipSuccess) return fail(FB_ENOMEM, "fb_check_views: device allocation failed");
    static const int kNone = INT_MAX;  // the initial value (a copy source that outlives the call)
    int first = INT_MAX, bad = 0;
    hipError_t e = hipMemcpyAsync(d, &kNone, sizeof(int), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) {
        k_check_views<<<(n_sel + 255) / 256, 256, 0, stream>>>(views, n_sel, p->g.n_views, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&first, d, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess && first != INT_MAX)
        e = hipMemcpy(&bad, views + first, sizeof(int32_t), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "fb_check_views");
    if (first != INT_MAX)
        return fail(FB_ESUBSET, "fb_check_views: views[" + std::to_string(first) + "] = " + std::to_string(bad) +
                                    " lies outside [0, " + std::to_string(p->g.n_views) + ")");
    return FB_OK;
}
