// The plain product y = A x / y = Aᵀ x without any allocation: its scratch
// (the launch descriptor, the launch list and, for the striped transposed
// product, the per-row-block partial vectors) lives in one fixed device
// array per GPU, so callers that cannot allocate device memory can use it.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "runtime.hpp"
#include "solve.hpp"

namespace plss {

// The array itself.  Host code never passes its name to a kernel or a copy:
// the name is a host-side stand-in, and every use goes through the device
// address looked up once per device (scratch_ptr).
static __device__ __align__(256) char scratch[PLSS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

struct DeviceSlot {
  std::once_flag once;
  hipError_t err = hipSuccess;
  char* ptr = nullptr;
  std::mutex mu;  // one product at a time per device: calls share the array
};

DeviceSlot g_slots[kMaxDevices];

// Fill the launch list of a plain product: (0, t) for t < count, or, for the
// striped transposed product, position kMaxBlk * q + b = (0, b << 24 | q)
// while block b has a unit q, else (0, -1).
struct UnitCounts {
  int v[kMaxBlk];
};

__global__ void k_fill_list(int2* __restrict__ l, int count, int striped_t, int nblk, UnitCounts nu) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    if (!striped_t) {
      l[i] = make_int2(0, i);
    } else {
      const int q = i / kMaxBlk, b = i % kMaxBlk;
      l[i] = make_int2(0, (b < nblk && q < nu.v[b]) ? ((b << 24) | q) : -1);
    }
  }
}

}  // namespace

// Look up this device's copy of the array (the device must be current).
// Called once per device from handle creation; the product looks it up too
// if a handle was made before the array existed.
char* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) throw InvalidArg{"device index beyond the scratch table"};
  DeviceSlot& s = g_slots[device];
  std::call_once(s.once, [&] {
    void* p = nullptr;
    s.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    s.ptr = static_cast<char*>(p);
  });
  if (s.err != hipSuccess || !s.ptr) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(s.err));
    throw DeviceError{};
  }
  return s.ptr;
}

static bool device_pointer(const void* p, int device) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice && a.device == device;
}

size_t spmv_noalloc_bytes(const plss_matrix* A, bool transpose, size_t* list_count) {
  const size_t o_list = align256(sizeof(Desc));
  size_t count = 0, ypart = 0;
  if (transpose ? (A->t_striped && !A->f32) : A->a_striped) {
    if (!transpose) {
      count = A->SA.nunits;
    } else {
      int qmax = 0;
      for (int b = 0; b < A->nblk; ++b) qmax = std::max(qmax, A->SB[b].nunits);
      count = (size_t)qmax * kMaxBlk;
      ypart = 8 * (size_t)A->nblk * (size_t)A->n;
    }
  } else {
    count = (transpose ? A->T : A->A).ntiles;
  }
  if (list_count) *list_count = count;
  return align256(o_list + sizeof(int2) * std::max<size_t>(1, count)) + ypart;
}

void spmv_noalloc(plss_handle* h, const plss_matrix* A, bool transpose, const double* x, double* y,
                  hipStream_t s) {
  const size_t nin = transpose ? A->m : A->n, nout = transpose ? A->n : A->m;
  if (!device_pointer(x, h->device) || !device_pointer(y, h->device))
    throw InvalidArg{"x and y must be device memory on the handle's GPU"};
  const char* xb = reinterpret_cast<const char*>(x);
  const char* yb = reinterpret_cast<const char*>(y);
  if (xb < yb + 8 * nout && yb < xb + 8 * nin) throw InvalidArg{"x and y overlap"};
  size_t count = 0;
  const size_t need = spmv_noalloc_bytes(A, transpose, &count);
  if (need > (size_t)PLSS_NOALLOC_SCRATCH_BYTES)
    throw InvalidArg{"the product needs " + std::to_string(need) + " bytes of scratch; the fixed array holds " +
                     std::to_string((size_t)PLSS_NOALLOC_SCRATCH_BYTES)};
  char* base = scratch_ptr(h->device);
  std::lock_guard<std::mutex> lk(g_slots[h->device].mu);

  Desc* dd = reinterpret_cast<Desc*>(base);
  int2* dl = reinterpret_cast<int2*>(base + align256(sizeof(Desc)));
  double* yp = reinterpret_cast<double*>(base + align256(align256(sizeof(Desc)) +
                                                         sizeof(int2) * std::max<size_t>(1, count)));
  Desc d;
  std::memset(&d, 0, sizeof(d));
  d.m = (int)A->m;
  d.n = (int)A->n;
  d.p = const_cast<double*>(x);
  d.r64 = y;
  const bool striped = transpose ? (A->t_striped && !A->f32) : A->a_striped;
  UnitCounts nu;
  std::memset(&nu, 0, sizeof(nu));
  if (striped) {
    if (!transpose) {
      fill_stripe_view(A->SA, &d.sa);
    } else {
      for (int b = 0; b < A->nblk; ++b) {
        fill_stripe_view(A->SB[b], &d.sb[b]);
        nu.v[b] = A->SB[b].nunits;
      }
      d.ypart = yp;
    }
  } else {
    d.a_ptr = A->A.ptr;
    d.a_idx = A->A.idx;
    d.a_val = A->A.val;
    d.a_tile = A->A.tile;
    d.a_ntiles = A->A.ntiles;
    d.a_nwt = A->A.nwt;
    d.a_grp = A->A.grp;
    d.a_wtd = A->A.wtd;
    d.t_ptr = A->T.ptr;
    d.t_idx = A->T.idx;
    d.t_val = A->T.val;
    d.t_tile = A->T.tile;
    d.t_ntiles = A->T.ntiles;
    d.t_nwt = A->T.nwt;
    d.t_grp = A->T.grp;
    d.t_wtd = A->T.wtd;
  }
  // the descriptor goes from this stack frame: the copy is complete once the
  // stream is synchronised below, before the frame ends
  PLSS_HIP(hipMemcpyAsync(dd, &d, sizeof(Desc), hipMemcpyHostToDevice, s));
  if (count > 0) {
    const int threads = 256;
    const int blocks = (int)std::min<size_t>((count + threads - 1) / threads, 4096);
    k_fill_list<<<blocks, threads, 0, s>>>(dl, (int)count, striped && transpose ? 1 : 0, A->nblk, nu);
    PLSS_HIP(hipGetLastError());
    if (striped) {
      launch_sspmv(MODE_PLAIN, A->f32, dd, dl, (int)count, transpose ? 1 : 0, s);
      if (transpose) st_ysum(yp, A->nblk, (int)A->n, y, s);
    } else {
      const PlssDir& dir = transpose ? A->T : A->A;
      launch_spmv(MODE_PLAIN, A->f32, dir.V, dd, dl, dir.ntiles, transpose ? 1 : 0, s);
    }
  } else if (nout > 0) {
    // no tiles or units (no entries): the product is zero
    PLSS_HIP(hipMemsetAsync(y, 0, 8 * nout, s));
  }
  PLSS_HIP(hipStreamSynchronize(s));
}

}  // namespace plss
