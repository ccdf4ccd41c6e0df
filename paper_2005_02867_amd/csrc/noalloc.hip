// Handle-free entry point that allocates nothing: the liquid volume
// h^3 sum(alpha) of a caller's cell array, reduced in the same fixed order as
// ds_droplet_volume reduces a handle's state.  Its only device memory beyond
// the caller's input and output is `scratch`, a file-scope array of this
// library (one copy per GPU, held until the process ends).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/dsvof.h"
#include "ds_device.h"
#include "ds_kernels.h"

using namespace dsv;

namespace {

// Scratch layout: one partial per block (at most MAX_BLOCKS blocks), then the
// completion counter of the last-block reduction on its own 256-byte line.
constexpr size_t kPartialBytes = (size_t)MAX_BLOCKS * sizeof(double);
constexpr size_t kCounterOff = kPartialBytes;
static_assert(DS_NOALLOC_SCRATCH_BYTES >= kCounterOff + 256, "scratch too small for its layout");

static __device__ __align__(256) unsigned char scratch[DS_NOALLOC_SCRATCH_BYTES];

// The volume sum of k_diagnostics (same block ranges, accumulation order and
// block reduction), written to a caller device scalar.
__global__ void k_volume_noalloc(const double* __restrict__ alpha, long long n, double h3, unsigned char* scr,
                                 double* out) {
  double* partials = reinterpret_cast<double*>(scr);
  unsigned* counter = reinterpret_cast<unsigned*>(scr + kCounterOff);
  long long b0, b1;
  block_range(n, b0, b1);
  double acc[1] = {0.0};
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) acc[0] += alpha[e];
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double tot[1];
    block_combine<1>(ops, partials, counter, tot);
    if (threadIdx.x == 0) *out = h3 * tot[0];
  }
}

// The counter must read zero when the reduction starts: a kernel clears it
// (no memset node, so the call can be captured into a graph).
__global__ void k_clear_counter(unsigned char* scr) {
  *reinterpret_cast<unsigned*>(scr + kCounterOff) = 0u;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` on each device, found once
thread_local std::string t_err;

int fail_noalloc(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

}  // namespace

// Message of the calling thread's last failed handle-free call.
const char* dsv_noalloc_last_error() { return t_err.c_str(); }

extern "C" int ds_droplet_volume_noalloc(const double* alpha, int nx, int ny, int nz, double h, double* m3,
                                         void* stream) {
  if (!alpha || !m3) return fail_noalloc(DS_ERR_ARG, "null pointer argument");
  if (nx < 1 || ny < 1 || nz < 1) return fail_noalloc(DS_ERR_ARG, "grid extents must be at least 1");
  const long long n = (long long)nx * ny * nz;
  if (n > DS_NOALLOC_MAX_CELLS)
    return fail_noalloc(DS_ERR_ARG, "grid of " + std::to_string(n) + " cells exceeds the maximum of " +
                                        std::to_string((long long)DS_NOALLOC_MAX_CELLS));
  if (!(h > 0.0)) return fail_noalloc(DS_ERR_ARG, "h must be positive");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail_noalloc(DS_ERR_HIP, "no current HIP device");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
      // the array's device address on this device (the current one); the
      // array's name in host code is only a stand-in for the symbol
      const hipError_t e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        g_scratch_ptr[dev] = nullptr;
        return fail_noalloc(DS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      }
    }
    ptr = g_scratch_ptr[dev];
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  unsigned char* scr = static_cast<unsigned char*>(ptr);
  k_clear_counter<<<1, 1, 0, s>>>(scr);
  k_volume_noalloc<<<grid_blocks(n), BLOCK, 0, s>>>(alpha, n, h * h * h, scr, m3);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_noalloc(DS_ERR_HIP, std::string("launch: ") + hipGetErrorString(e));
  t_err.clear();
  return DS_OK;
}
