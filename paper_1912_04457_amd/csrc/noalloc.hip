// Collision term without a context and without device allocation: the
// buffers that qgbe_init_grid would allocate (channel table and lists,
// masses and their partial sums, per-launch totals, the FP32 shadow of f and
// its node quads) are carved out of one statically sized device array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "context.h"

using namespace qgbe;

namespace {

constexpr size_t kScratchBytes = size_t(QGBE_NOALLOC_SCRATCH_MIB) << 20;
constexpr int kMaxDevices = 64;

// One copy per GPU.  Host code never uses this name as an address: it takes
// the device address from hipGetSymbolAddress once per device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceState {
  bool ready = false;
  unsigned char* ptr = nullptr;   // this device's copy of scratch
  size_t lds[3] = {0, 0, 0};      // dynamic LDS budgets of the FP32 kernels
  int n_cu = 256;
  // what the channel-table region holds (host copy of the last upload)
  std::vector<unsigned char> table;
};

std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Once per device, with that device current.
qgbe_status setup(int device, DeviceState** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState& s = g_dev[device];
  if (!s.ready) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address");
    int lds_max = 0;
    HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device), "query LDS size");
    HIP_TRY(set_collide_lds_limit((size_t)std::max(lds_max, 0), &s.lds[0], &s.lds[1], &s.lds[2]),
            "raise the dynamic LDS limit");
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && n_cu > 0)
      s.n_cu = n_cu;
    s.ptr = static_cast<unsigned char*>(p);
    s.ready = true;
  }
  *out = &s;
  return QGBE_OK;
}

// Bump allocation inside the scratch array.
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <typename T>
  T* take(size_t n) {
    T* p = reinterpret_cast<T*>(base + used);
    used += align256(n * sizeof(T));
    return p;
  }
};

}  // namespace

extern "C" {

size_t qgbe_noalloc_scratch_bytes(void) { return kScratchBytes; }

qgbe_status qgbe_collision_term_noalloc(const qgbe_grid_desc* desc, const double* f, uint32_t step,
                                        int32_t n_samples, int32_t sampler, double* A) {
  if (!f || !A) return fail(QGBE_EINVAL, "NULL argument");
  qgbe_status st = validate(desc);
  if (st) return st;
  if (n_samples < 1) return fail(QGBE_EINVAL, "n_samples must be >= 1");
  if (sampler != QGBE_SAMPLER_UNIFORM && sampler != QGBE_SAMPLER_ROOTS && sampler != QGBE_SAMPLER_ROOTS_ALT)
    return fail(QGBE_EINVAL, "sampler must be uniform or one of the root samplers (no proposal table here)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(QGBE_EDEVICE, "no HIP device");
  if (desc->device < 0 || desc->device >= std::min(ndev, kMaxDevices))
    return fail(QGBE_EINVAL, "device ordinal out of range");
  HIP_TRY(hipSetDevice(desc->device), "hipSetDevice");
  DeviceState* dev = nullptr;
  st = setup(desc->device, &dev);
  if (st) return st;

  // A context on the stack: the launch plan of qgbe_init_grid, with every
  // device buffer inside scratch.
  qgbe_ctx c;
  c.d = *desc;
  c.stream = (hipStream_t)desc->stream;
  make_grid(desc, c.G);
  c.chans.resize(kMaxChannels);
  c.nch = build_channels(desc->species_mask, desc->row_mask, c.chans.data(), kMaxChannels);
  c.chans.resize(c.nch);
  c.lds_budget[0] = dev->lds[0];
  c.lds_budget[1] = dev->lds[1];
  c.lds_budget_queue = dev->lds[2];
  c.n_cu = dev->n_cu;
  c.step = step;
  plan_groups(&c);

  const size_t n = field_len(&c);
  const int nch1 = std::max(1, c.nch);
  const bool fp32 = desc->precision == QGBE_FP32 && sampler == QGBE_SAMPLER_UNIFORM;
  Carve cv{dev->ptr};
  c.d_chans = cv.take<Channel>(kMaxChannels);
  c.d_groups = cv.take<int>(kMaxChannels);
  c.d_all = cv.take<int>(kMaxChannels);
  const size_t table_bytes = cv.used;
  c.d_mass2 = cv.take<double>((size_t)kSpecies * c.G.cells);
  c.d_mass_part = cv.take<double>(mass_scratch(c.G));
  c.d_count = cv.take<unsigned long long>(kStripes);
  c.d_mc = cv.take<double>(2 * kStripes);
  c.d_chan_var = cv.take<double>((size_t)kStripes * nch1);
  if (fp32) {
    c.d_f32 = cv.take<float>(n);
    if (c.need_quads[0]) c.d_f32q = cv.take<float4>(n);
  }
  if (cv.used > kScratchBytes)
    return fail(QGBE_EINVAL, "grid needs " + std::to_string(cv.used) + " bytes of scratch, more than the " +
                                 std::to_string(kScratchBytes) + " of qgbe_collision_term_noalloc");
  c.d_f = const_cast<double*>(f);  // read only: masses and the collision kernels

  // Channel table, group lists and identity list, uploaded when they differ
  // from what this device's scratch holds and waited for; the host record of
  // what the scratch holds changes only after the upload has completed, so a
  // failed upload is retried by the next call.
  std::vector<unsigned char> tab(table_bytes, 0);
  std::memcpy(tab.data(), c.chans.data(), c.chans.size() * sizeof(Channel));
  std::memcpy(tab.data() + ((unsigned char*)c.d_groups - dev->ptr), c.group_index.data(),
              c.group_index.size() * sizeof(int));
  int* all = reinterpret_cast<int*>(tab.data() + ((unsigned char*)c.d_all - dev->ptr));
  for (int i = 0; i < c.nch; ++i) all[i] = i;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (dev->table != tab) {
      dev->table.clear();
      HIP_TRY(hipMemcpyAsync(dev->ptr, tab.data(), table_bytes, hipMemcpyHostToDevice, c.stream),
              "copy channel table");
      HIP_TRY(hipStreamSynchronize(c.stream), "synchronise");
      dev->table = std::move(tab);
    }
  }

  st = compute_masses(&c);
  if (st) return st;
  if (fp32) HIP_TRY(launch_to_f32(c.d_f, c.d_f32, n, c.stream), "f to fp32");
  HIP_TRY(launch_fill(A, 0.0, n, c.stream), "zero A");
  return run_collide(&c, n_samples, sampler, A, nullptr, nullptr);
}

}  // extern "C"
