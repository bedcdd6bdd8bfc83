// gs2d_image_loss_noalloc: the masked L1 image loss of gs2d_image_loss without a
// context and without any allocation.  Its scratch memory (the one-view descriptor
// table and the per-workgroup partial sums) is a file-scope device array of fixed
// size; every GPU the library runs on holds its own copy until the process ends.
//
// Host code never passes the array's name to a kernel (in host code the name is a
// host-side stand-in, not a device address).  The first call on a device, with that
// device current, looks up the array's device address with hipGetSymbolAddress and
// keeps it per device; every launch takes that address.
#include <mutex>

#include <cmath>
#include <cstring>

#include "pose_step.h"

namespace gs2d {
namespace {

constexpr int64_t kNoAllocMaxPixels = GS2D_NOALLOC_MAX_PIXELS;
constexpr size_t kViewSlotBytes = 1024;  // the one-view descriptor table
constexpr size_t kPartBytes = (size_t)((kNoAllocMaxPixels + kLossThreads - 1) / kLossThreads) * sizeof(float);
constexpr int kMaxDevices = 64;
static_assert(sizeof(ViewDesc) <= kViewSlotBytes, "view descriptor slot too small");

// descriptor table at offset 0, partial sums at kViewSlotBytes
static __device__ __align__(256) unsigned char scratch[kViewSlotBytes + kPartBytes];

std::mutex g_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (looked up once per device).
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return GS2D_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GS2D_ERR_HIP;
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return GS2D_OK;
}

}  // namespace
}  // namespace gs2d

extern "C" {

GS2D_API int gs2d_image_loss_noalloc(const gs2d_camera* camera, const float* rgb, const float* depth,
                                     const float* normal, const float* alpha, const float* tgt_rgb,
                                     const float* tgt_depth, const float* tgt_normal, const gs2d_loss_weights* w,
                                     float* loss, float* d_rgb, float* d_depth, float* d_normal, hipStream_t stream) {
  using namespace gs2d;
  if (!camera || camera->width <= 0 || camera->height <= 0 || !(camera->fx > 0.f) || !(camera->fy > 0.f) ||
      !std::isfinite(camera->cx) || !std::isfinite(camera->cy) || !w || !loss || !depth || !tgt_depth)
    return GS2D_ERR_INVALID_ARG;
  if (!std::isfinite(w->w_rgb) || !std::isfinite(w->w_depth) || !std::isfinite(w->w_normal))
    return GS2D_ERR_INVALID_ARG;
  if ((w->w_rgb != 0.f || d_rgb) && (!rgb || !tgt_rgb)) return GS2D_ERR_INVALID_ARG;
  if ((w->w_normal != 0.f || d_normal) && (!normal || !tgt_normal)) return GS2D_ERR_INVALID_ARG;
  if ((w->normal_mask && !normal) || (w->opacity_mask && !alpha)) return GS2D_ERR_INVALID_ARG;
  const int64_t hw64 = (int64_t)camera->width * camera->height;
  if (hw64 > kNoAllocMaxPixels) return GS2D_ERR_CAPACITY;
  const int hw = (int)hw64;
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess) return GS2D_ERR_HIP;
  unsigned char* base = nullptr;
  const int r = scratch_address(device, &base);
  if (r != GS2D_OK) return r;
  ViewDesc* views = reinterpret_cast<ViewDesc*>(base);
  float* part = reinterpret_cast<float*>(base + kViewSlotBytes);
  ViewSet vs;
  vs.n_views = 1;
  ViewDesc& d = vs.v[0];
  std::memset(&d, 0, sizeof(d));
  d.cam = CamF{camera->width, camera->height, camera->fx, camera->fy, camera->cx, camera->cy};
  const bool colour = w->w_rgb != 0.f || d_rgb, normals = w->w_normal != 0.f || d_normal;
  d.rgb = colour ? const_cast<float*>(rgb) : nullptr;
  d.tgt_rgb = colour ? tgt_rgb : nullptr;
  d.depth = const_cast<float*>(depth);
  d.tgt_depth = tgt_depth;
  d.normal = const_cast<float*>(normal);
  d.tgt_normal = normals ? tgt_normal : nullptr;
  d.alpha = const_cast<float*>(alpha);
  d.g_rgb = d_rgb;
  d.g_depth = d_depth;
  d.g_normal = d_normal;
  // every partial the reduction reads is written by this call's loss kernel, and the
  // descriptor by its upload: nothing has to start at zero
  launch_upload_views(vs, views, stream);
  launch_image_loss(views, 1, hw, LossW{w->w_rgb, w->w_depth, w->w_normal, w->normal_mask, w->opacity_mask}, part,
                    loss_blocks(hw), stream);
  launch_reduce_loss(part, loss_blocks(hw), 1.0f / (float)hw, loss, stream);
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_ERR_HIP;
}

}  // extern "C"
