// tt_noalloc.hip -- the allocation-free form of the diagnostic Cholesky solve, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving loops).
//
// Every workspace the factorisation and the back substitution need (the padded working matrix with
// its right-hand-side row, the inverse diagonal blocks, the hand-over flags, the scalars, the
// tagged substitution entries, the scaling and the solution) lives in one file-scope device array,
// `scratch`, of TT_NOALLOC_SCRATCH_BYTES per GPU. Host code never passes the array's name to a
// kernel (on the host it only names a stand-in): the first call on a device resolves the device
// address with hipGetSymbolAddress, with that device current, and keeps it per device. All set-up
// runs in kernels (no memset or copy nodes), so a caller may capture the call into a graph.
#include <mutex>

#include "tt_internal.h"

namespace {

constexpr int kMaxN = TT_NOALLOC_MAX_N;
constexpr int kMaxPad = ((kMaxN + TT_NB - 1) / TT_NB) * TT_NB;
constexpr int kMaxNb = kMaxPad / TT_NB;

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Byte offsets of the regions, each sized for n = kMaxN and aligned to 256 bytes.
constexpr size_t kOffA = 0;
constexpr size_t kOffLinv = kOffA + align256(sizeof(float) * (size_t)(kMaxPad + TT_NB) * kMaxPad);
constexpr size_t kOffFlags = kOffLinv + align256(sizeof(float) * (size_t)kMaxNb * TT_NB * TT_NB);
constexpr size_t kFlagInts = (size_t)kMaxNb + (size_t)(kMaxNb + 1) * kMaxNb + 4 * (size_t)kMaxNb + 2;
constexpr size_t kOffSc = kOffFlags + align256(sizeof(int) * kFlagInts);
constexpr size_t kOffTw = kOffSc + align256(sizeof(LMScalars));
constexpr size_t kOffScale = kOffTw + align256(sizeof(uint64_t) * kMaxPad);
constexpr size_t kOffX = kOffScale + align256(sizeof(float) * kMaxPad);
constexpr size_t kBytes = kOffX + align256(sizeof(float) * kMaxPad);
static_assert(kBytes == TT_NOALLOC_SCRATCH_BYTES, "tt.h states the scratch size");

static __device__ __align__(256) unsigned char scratch[kBytes];

// Padded working matrix (ld = npad): the lower triangle of A, an identity on the padding, b in the
// first right-hand-side row, zero elsewhere; unit scaling, cleared flags and tagged entries, and
// scalars set for one solve of epoch 1.
__global__ void k_noalloc_setup(float* __restrict__ Ap, const float* __restrict__ A, const float* __restrict__ b,
                                int n, int npad, float* __restrict__ dscale, int* __restrict__ flags, int nflags,
                                uint64_t* __restrict__ tw, LMScalars* sc) {
  const size_t total = (size_t)(npad + TT_NB) * npad;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += stride) {
    const int r = (int)(e / npad), c = (int)(e % npad);
    float v = 0.0f;
    if (r < n && c <= r) v = A[(size_t)r * n + c];
    else if (r >= n && r < npad && c == r) v = 1.0f;
    else if (r == npad && c < n) v = b[c];
    Ap[e] = v;
  }
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)npad; e += stride) {
    dscale[e] = 1.0f;
    tw[e] = 0ull;
  }
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < (size_t)nflags; e += stride) flags[e] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->lambda = 0.0;
    sc->e_old = 0.0;
    sc->e_new = 0.0;
    sc->w_arap = 0.0;
    sc->sum_omega = 0.0;
    sc->sum_orbw = 0.0;
    sc->eps = 0.0;
    sc->chol_fail = 0;
    sc->accept = 0;
    sc->it = 0;
    sc->err = 0;
    sc->solve_epoch = 1;
  }
}

__global__ void k_noalloc_finish(const float* __restrict__ xs, float* __restrict__ x, int n,
                                 const LMScalars* __restrict__ sc, int32_t* __restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = xs[i];
  if (i == 0) {
    status[0] = sc->chol_fail;
    status[1] = sc->err;
  }
}

struct DevScratch {
  void* ptr = nullptr;
  int cus = 0, wall_khz = 0;
};
constexpr int kMaxDevices = 64;
std::mutex g_mu;
DevScratch g_dev[kMaxDevices];

// The device address of `scratch` on the current device (resolved once per device).
int scratch_for_current_device(DevScratch* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TT_EDEVICE;
  std::lock_guard<std::mutex> g(g_mu);
  DevScratch& s = g_dev[dev];
  if (!s.ptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TT_EDEVICE;
    int cus = 0, khz = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return TT_EDEVICE;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return TT_EDEVICE;
    s.cus = cus;
    s.wall_khz = khz;
    s.ptr = p;
  }
  *out = s;
  return TT_OK;
}

}  // namespace

extern "C" int tt_cholesky_solve_noalloc(int n, const float* d_A, const float* d_b, float* d_x, int32_t* d_status,
                                         void* hip_stream) {
  if (n < 1 || n > kMaxN || !d_A || !d_b || !d_x || !d_status) return TT_EINVAL;
  DevScratch ds;
  int rc = scratch_for_current_device(&ds);
  if (rc) return rc;
  unsigned char* base = static_cast<unsigned char*>(ds.ptr);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  DevState d;
  d.n = n;
  d.npad = ((n + TT_NB - 1) / TT_NB) * TT_NB;
  d.nb = d.npad / TT_NB;
  d.ld = d.npad;
  d.prec = TT_FP32;
  d.ir_iters = 0;
  d.num_cus = ds.cus;
  d.wall_khz = ds.wall_khz;
  d.A = reinterpret_cast<float*>(base + kOffA);
  d.Linv = reinterpret_cast<float*>(base + kOffLinv);
  d.flags = reinterpret_cast<int*>(base + kOffFlags);
  d.sc = reinterpret_cast<LMScalars*>(base + kOffSc);
  d.tw = reinterpret_cast<uint64_t*>(base + kOffTw);
  d.dscale = reinterpret_cast<float*>(base + kOffScale);
  d.x = reinterpret_cast<float*>(base + kOffX);
  const int nflags = (int)chol_flag_ints(d.nb);
  hipLaunchKernelGGL(k_noalloc_setup, dim3(256), dim3(256), 0, st, d.A, d_A, d_b, n, d.npad, d.dscale, d.flags,
                     nflags, d.tw, d.sc);
  if (hipGetLastError() != hipSuccess) return TT_EDEVICE;
  if (launch_cholesky_factor(d, st) != hipSuccess) return TT_EDEVICE;
  if (launch_cholesky_backsolve(d, 0, st) != hipSuccess) return TT_EDEVICE;
  hipLaunchKernelGGL(k_noalloc_finish, dim3((n + 255) / 256), dim3(256), 0, st, d.x, d_x, n, d.sc, d_status);
  return hipGetLastError() == hipSuccess ? TT_OK : TT_EDEVICE;
}
