// Both products of one residual-sketch iteration (Algorithm 1: r <- r - A p,
// then y = Aᵀ r with the updated r) in one pass over the CSR store of A, with
// a deterministic two-level sum for y:
//   level 1 (k_fz_rows): each row's dot a_iᵀp, the residual update, and the
//     row's contributions c_e = a_e r_i written in CSR order;
//   level 2 (k_fz_cols): y_j = sum of column j's contributions, read through
//     the CSR position of each CSC slot (rows ascending), in a fixed order.
// Groups of 16 lanes own one row of at most 64 entries (one column); a whole
// wave owns each longer row.  Every sum has a fixed order (lane-strided
// partials, then a butterfly over the lanes, then a fixed sequence over
// waves, groups and workgroups), so results are bit-reproducible.
#include "fused.hpp"

#include <algorithm>

namespace plss {

namespace {

constexpr int kFzLanes = 16;              // lanes per row / column
constexpr int kFzGroups = kWG / kFzLanes;  // rows per workgroup at a time
constexpr int kFzShort = 64;               // longer rows are the matrix's long-row list

// sum over the 16 lanes of a group; every lane ends with the same value
// (each butterfly step adds the same two operands in both lanes)
__device__ inline double sum16(double v) {
  v += __shfl_xor(v, 8, kFzLanes);
  v += __shfl_xor(v, 4, kFzLanes);
  v += __shfl_xor(v, 2, kFzLanes);
  v += __shfl_xor(v, 1, kFzLanes);
  return v;
}

// per-workgroup sum of the groups' values (lane 0 of each group), fixed order
__device__ inline void block_part(double v, double* part) {
  __shared__ double s[kFzGroups];
  const int sl = threadIdx.x % kFzLanes, g = threadIdx.x / kFzLanes;
  if (sl == 0) s[g] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kFzGroups; ++q) t += s[q];
    part[blockIdx.x] = t;
  }
}

template <class Val>
__global__ __launch_bounds__(kWG) void k_fz_rows(const int* __restrict__ ptr, const int* __restrict__ idx,
                                                 const Val* __restrict__ val, int m, const double* __restrict__ p,
                                                 double* __restrict__ r, double* __restrict__ c,
                                                 double* __restrict__ part) {
  const int sl = threadIdx.x % kFzLanes, g = threadIdx.x / kFzLanes;
  const int stride = gridDim.x * kFzGroups;
  double rr = 0.0;
  for (int i = blockIdx.x * kFzGroups + g; i < m; i += stride) {
    const int e0 = ptr[i], e1 = ptr[i + 1];
    if (e1 - e0 > kFzShort) continue;  // k_fz_long
    double acc = 0.0;
    for (int e = e0 + sl; e < e1; e += kFzLanes) acc += (double)val[e] * p[idx[e]];
    acc = sum16(acc);
    const double ri = r[i] - acc;
    for (int e = e0 + sl; e < e1; e += kFzLanes) c[e] = (double)val[e] * ri;
    if (sl == 0) {
      r[i] = ri;
      rr += ri * ri;
    }
  }
  block_part(rr, part);
}

// rows of more than kFzShort entries (the ascending list lrows), one wave
// per row: four entries per lane in flight, then the fixed-order butterfly
// over the 64 lanes; the four waves' partial rho in wave order
template <class Val>
__global__ __launch_bounds__(kWG) void k_fz_long(const int* __restrict__ ptr, const int* __restrict__ idx,
                                                 const Val* __restrict__ val, const int* __restrict__ lrows,
                                                 int nlong, const double* __restrict__ p, double* __restrict__ r,
                                                 double* __restrict__ c, double* __restrict__ part) {
  __shared__ double s_w[kWG / 64];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int stride = gridDim.x * (kWG / 64);
  double rr = 0.0;
  for (int q = blockIdx.x * (kWG / 64) + w; q < nlong; q += stride) {
    const int i = lrows[q];
    const int e0 = ptr[i], e1 = ptr[i + 1];
    const double r_old = r[i];
    double acc = 0.0;
    int e = e0 + lane;
    for (; e + 3 * 64 < e1; e += 4 * 64) {
      const Val v0 = val[e], v1 = val[e + 64], v2 = val[e + 128], v3 = val[e + 192];
      const int j0 = idx[e], j1 = idx[e + 64], j2 = idx[e + 128], j3 = idx[e + 192];
      const double p0 = p[j0], p1 = p[j1], p2 = p[j2], p3 = p[j3];
      acc += (double)v0 * p0;
      acc += (double)v1 * p1;
      acc += (double)v2 * p2;
      acc += (double)v3 * p3;
    }
    for (; e < e1; e += 64) acc += (double)val[e] * p[idx[e]];
    for (int o = 32; o > 0; o /= 2) acc += __shfl_xor(acc, o, 64);
    const double ri = r_old - acc;
    for (int f = e0 + lane; f < e1; f += 64) c[f] = (double)val[f] * ri;
    if (lane == 0) {
      r[i] = ri;
      rr += ri * ri;
    }
  }
  if (lane == 0) s_w[w] = rr;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int v = 0; v < kWG / 64; ++v) t += s_w[v];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kWG) void k_fz_cols(const int* __restrict__ cptr, const int* __restrict__ pos,
                                                 const double* __restrict__ c, int n, double* __restrict__ y,
                                                 double* __restrict__ part) {
  const int sl = threadIdx.x % kFzLanes, g = threadIdx.x / kFzLanes;
  const int stride = gridDim.x * kFzGroups;
  double yy = 0.0;
  for (int j = blockIdx.x * kFzGroups + g; j < n; j += stride) {
    const int k0 = cptr[j], k1 = cptr[j + 1];
    double acc = 0.0;
    int k = k0 + sl;
    for (; k + 3 * kFzLanes < k1; k += 4 * kFzLanes) {
      const int q0 = pos[k], q1 = pos[k + kFzLanes], q2 = pos[k + 2 * kFzLanes], q3 = pos[k + 3 * kFzLanes];
      const double c0 = c[q0], c1 = c[q1], c2 = c[q2], c3 = c[q3];
      acc += c0;
      acc += c1;
      acc += c2;
      acc += c3;
    }
    for (; k < k1; k += kFzLanes) acc += c[pos[k]];
    acc = sum16(acc);
    if (sl == 0) {
      y[j] = acc;
      yy += acc * acc;
    }
  }
  block_part(yy, part);
}

// out[0] = sum of a[0..na), out[1] = sum of b[0..nb), each in a fixed order
__global__ __launch_bounds__(kWG) void k_fz_fin(const double* __restrict__ a, int na, const double* __restrict__ b,
                                                int nb, double* __restrict__ out) {
  __shared__ double s[2][kWG];
  double ta = 0.0, tb = 0.0;
  for (int q = threadIdx.x; q < na; q += kWG) ta += a[q];
  for (int q = threadIdx.x; q < nb; q += kWG) tb += b[q];
  s[0][threadIdx.x] = ta;
  s[1][threadIdx.x] = tb;
  __syncthreads();
  for (int w = kWG / 2; w > 0; w /= 2) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s[0][0];
    out[1] = s[1][0];
  }
}

// pos[k] = CSR position of CSC slot k: column j's slots hold its rows in
// ascending order, and row i's columns are ascending and distinct in the
// CSR, so a binary search of row i finds entry (i, j)
__global__ __launch_bounds__(kWG) void k_fz_pos(const int* __restrict__ aptr, const int* __restrict__ aidx,
                                                const int* __restrict__ cptr, const int* __restrict__ ridx, int n,
                                                int* __restrict__ pos) {
  const int sl = threadIdx.x % kFzLanes, g = threadIdx.x / kFzLanes;
  const int stride = gridDim.x * kFzGroups;
  for (int j = blockIdx.x * kFzGroups + g; j < n; j += stride) {
    for (int k = cptr[j] + sl; k < cptr[j + 1]; k += kFzLanes) {
      const int i = ridx[k];
      int lo = aptr[i], hi = aptr[i + 1];
      const int last = hi - 1;
      while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (aidx[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      pos[k] = lo <= last ? lo : max(last, 0);  // the entry exists: lo is its position
    }
  }
}

}  // namespace

int fz_grid(long long rows) {
  const long long g = (rows + kFzGroups - 1) / kFzGroups;
  return (int)std::max(1LL, std::min(g, (long long)kFzMaxGrid));
}

void launch_fz_pos(const int* aptr, const int* aidx, const int* cptr, const int* ridx, int n, int* pos,
                   hipStream_t s) {
  k_fz_pos<<<fz_grid(n), kWG, 0, s>>>(aptr, aidx, cptr, ridx, n, pos);
  PLSS_HIP(hipGetLastError());
}

int fz_long_grid(int nlong) { return nlong > 0 ? std::min((nlong + kWG / 64 - 1) / (kWG / 64), kFzMaxGrid) : 0; }

void launch_fz_pair(bool f32, const int* ptr, const int* idx, const void* val, int m, const int* lrows,
                    int nlong, const int* cptr, const int* pos, int n, const double* p, double* r, double* c,
                    double* y, double* part, double* out2, hipStream_t s) {
  const int g1 = fz_grid(m), gl = fz_long_grid(nlong), g2 = fz_grid(n);
  if (f32) {
    const float* v = static_cast<const float*>(val);
    k_fz_rows<float><<<g1, kWG, 0, s>>>(ptr, idx, v, m, p, r, c, part);
    if (gl) k_fz_long<float><<<gl, kWG, 0, s>>>(ptr, idx, v, lrows, nlong, p, r, c, part + g1);
  } else {
    const double* v = static_cast<const double*>(val);
    k_fz_rows<double><<<g1, kWG, 0, s>>>(ptr, idx, v, m, p, r, c, part);
    if (gl) k_fz_long<double><<<gl, kWG, 0, s>>>(ptr, idx, v, lrows, nlong, p, r, c, part + g1);
  }
  k_fz_cols<<<g2, kWG, 0, s>>>(cptr, pos, c, n, y, part + g1 + gl);
  k_fz_fin<<<1, kWG, 0, s>>>(part, g1 + gl, part + g1 + gl, g2, out2);
  PLSS_HIP(hipGetLastError());
}

}  // namespace plss
