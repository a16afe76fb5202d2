// Velocity-conditioned scalar mean <phi|V> for eq:IECM on gfx950 (Ch.3, Sec.
// Estimation of the velocity-conditioned scalar mean; App. B).
//
// In every element the particles, starting from increasing id, are sorted by
// U and divided into cond_nu groups, each group by V into cond_nv, each by W
// into cond_nw; ties go by id, a direction with one interval is skipped, and a
// level is taken only while every subgroup keeps cond_min particles.  With P
// groups over the n particles of an element, the particle at position j of
// the order is in group P*j/n (the App. B bin index), so group g spans the
// positions [ceil(g n / P), ceil((g+1) n / P)).  A particle's <phi|V> is the
// mean psi of its final subgroup, summed in FP64 in the order of the positions.
//
// Every sort is a rank count within the group: the rank of a particle is the
// number of group members before it in (key, id) order, which is a
// permutation because ids are unique and the keys are compared as integers
// (an order-preserving map of the float bits, with -0 taken as +0).
//
// Launch sequence: count the particles per element (wave-aggregated atomics),
// scan, list the particles of every element; one 64-thread workgroup per
// element with at most 256 particles, all staged in LDS; elements with more go
// to a list that 256-thread workgroups work through in global memory, with
// LDS tiles for the rank counts.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "pdf_internal.h"

namespace pdfk {

namespace {

constexpr int CW = 256;  // particles of an element handled in LDS by one wave
constexpr int BT = 256;  // threads of the large-element workgroups

__device__ __forceinline__ uint64_t ordkey(float v) {
  const uint32_t b = __float_as_uint(v + 0.0f);  // -0 -> +0
  return (b & 0x80000000u) ? (uint64_t)(~b) : (uint64_t)(b | 0x80000000u);
}
__device__ __forceinline__ uint64_t ordkey(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v + 0.0);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

template <typename T>
__device__ __forceinline__ uint64_t level_key(const PartDev<T> &p, int dir, int32_t i) {
  if (dir < 0) return 0;  // the starting order: by id alone
  const T v = dir == 0 ? p.u[i] : (dir == 1 ? p.v[i] : p.w[i]);
  return ordkey(v);
}

// the passes of an element of n particles: directions dir[0..npass) with the
// group counts after each; with no level taken, one pass by id
struct Passes {
  int n_pass;
  int dir[3];
  int32_t groups[3];
};

__device__ __forceinline__ Passes plan_passes(const ModelDev &md, int32_t n) {
  const int32_t f[3] = {md.cond_nu, md.cond_nv, md.cond_nw};
  Passes ps;
  ps.n_pass = 0;
  int32_t nc = 1;
  for (int d = 0; d < 3; ++d) {
    if (f[d] <= 1) continue;
    const int32_t next = nc * f[d];
    if (n / next < md.cond_min) break;  // the adaptive stop
    ps.dir[ps.n_pass] = d;
    ps.groups[ps.n_pass] = next;
    ps.n_pass++;
    nc = next;
  }
  if (ps.n_pass == 0) {
    ps.n_pass = 1;
    ps.dir[0] = -1;
    ps.groups[0] = 1;
  }
  return ps;
}

__device__ __forceinline__ int32_t gstart(int64_t g, int64_t n, int64_t P) { return (int32_t)((g * n + P - 1) / P); }

// run-length aggregation of equal element numbers over a wave (particles are
// mostly sorted by element): a run is a stretch of valid lanes with the same
// element; returns the first lane of the caller's run (-1 for an invalid lane)
// and, for that first lane, the run length
__device__ __forceinline__ void wave_runs(int32_t e, bool valid, int &head_lane, int &len) {
  const int lane = threadIdx.x & 63;
  const int32_t prev = __shfl_up(e, 1, 64);
  const bool prev_valid = __shfl_up((int)valid, 1, 64) != 0;
  const bool head = valid && (lane == 0 || !prev_valid || prev != e);
  const uint64_t heads = __ballot(head);
  const uint64_t stops = heads | __ballot(!valid);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  head_lane = valid ? 63 - __clzll((long long)(heads & upto)) : -1;
  const uint64_t later = stops & ~upto;
  const int end = later ? __ffsll((unsigned long long)later) - 1 : 64;
  len = end - lane;
}

__global__ __launch_bounds__(256) void k_cond_count(int64_t np, int32_t ne, const int32_t *pe, int32_t *cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t e = i < np ? pe[i] : -1;
  const bool valid = e >= 0 && e < ne;
  int hl, len;
  wave_runs(e, valid, hl, len);
  if (hl == (int)(threadIdx.x & 63)) atomicAdd(&cnt[e], len);
}

__global__ __launch_bounds__(256) void k_cond_fill(int64_t np, int32_t ne, const int32_t *pe, const int32_t *off,
                                                   int32_t *cursor, int32_t *list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t e = i < np ? pe[i] : -1;
  const bool valid = e >= 0 && e < ne;
  int hl, len;
  wave_runs(e, valid, hl, len);
  const int lane = threadIdx.x & 63;
  int32_t base = 0;
  if (hl == lane) base = atomicAdd(&cursor[e], len);
  base = __shfl(base, hl < 0 ? lane : hl, 64);
  if (valid) list[off[e] + base + (lane - hl)] = (int32_t)i;
}

// one element of at most CW particles per 64-thread workgroup, in LDS
template <typename T>
__global__ __launch_bounds__(64) void k_cond_wave(int32_t ne, ModelDev md, PartDev<T> p, const int32_t *cnt,
                                                  const int32_t *off, const int32_t *list, int32_t *big,
                                                  int32_t *nbig, T *cm) {
  __shared__ uint64_t kp[CW];
  __shared__ uint32_t ip[2][CW];
  __shared__ int32_t sp[2][CW];
  const int32_t e = blockIdx.x;
  if (e >= ne) return;
  const int32_t n = cnt[e];
  if (n == 0) return;
  const int t = threadIdx.x;
  if (n > CW) {
    if (t == 0) big[atomicAdd(nbig, 1)] = e;
    return;
  }
  const int32_t base = off[e];
  for (int q = t; q < n; q += 64) {
    const int32_t i = list[base + q];
    sp[0][q] = i;
    ip[0][q] = p.id[i];
  }
  const Passes ps = plan_passes(md, n);
  int cur = 0;
  int32_t nc = 1;
  for (int pass = 0; pass < ps.n_pass; ++pass) {
    for (int q = t; q < n; q += 64) kp[q] = level_key(p, ps.dir[pass], sp[cur][q]);
    __syncthreads();
    for (int q = t; q < n; q += 64) {
      const int32_t g = (int32_t)((int64_t)nc * q / n);
      const int32_t s0 = gstart(g, n, nc), s1 = gstart(g + 1, n, nc);
      const uint64_t mk = kp[q];
      const uint32_t mid = ip[cur][q];
      int32_t rank = 0;
      for (int32_t r = s0; r < s1; ++r) {
        const uint64_t k = kp[r];
        const uint32_t id = ip[cur][r];
        // (key, id) order; the position breaks ties of equal ids, so the
        // ranks are a permutation whatever the input
        rank += (k < mk) | ((k == mk) & ((id < mid) | ((id == mid) & (r < q))));
      }
      sp[1 - cur][s0 + rank] = sp[cur][q];
      ip[1 - cur][s0 + rank] = mid;
    }
    __syncthreads();
    cur = 1 - cur;
    nc = ps.groups[pass];
  }
  // bin means (App. B), each bin summed in the order of its positions
  for (int32_t b = t; b < nc; b += 64) {
    const int32_t s0 = gstart(b, n, nc), s1 = gstart(b + 1, n, nc);
    double sum = 0.0;
    for (int32_t r = s0; r < s1; ++r) sum += (double)p.psi[sp[cur][r]];
    const T mean = (T)(sum / (double)(s1 - s0));
    for (int32_t r = s0; r < s1; ++r) cm[sp[cur][r]] = mean;
  }
}

// elements of more than CW particles: one 256-thread workgroup each, the
// order held in global memory (list <-> list2), the rank counts over LDS tiles
template <typename T>
__global__ __launch_bounds__(BT) void k_cond_block(ModelDev md, PartDev<T> p, const int32_t *cnt,
                                                   const int32_t *off, int32_t *list, int32_t *list2,
                                                   const int32_t *big, const int32_t *nbig, T *cm) {
  __shared__ uint64_t tk[BT];
  __shared__ uint32_t tid[BT];
  const int32_t nb = *nbig;
  const int t = threadIdx.x;
  for (int32_t k = blockIdx.x; k < nb; k += gridDim.x) {
    const int32_t e = big[k];
    const int32_t n = cnt[e];
    int32_t *A = list + off[e];
    int32_t *B = list2 + off[e];
    const Passes ps = plan_passes(md, n);
    int32_t nc = 1;
    for (int pass = 0; pass < ps.n_pass; ++pass) {
      const int dir = ps.dir[pass];
      for (int32_t c0 = 0; c0 < n; c0 += BT) {
        const int32_t q = c0 + t;
        const int32_t qlast = (c0 + BT < n ? c0 + BT : n) - 1;
        // the positions the groups of this chunk span
        const int32_t lo = gstart((int64_t)nc * c0 / n, n, nc);
        const int32_t hi = gstart((int64_t)nc * qlast / n + 1, n, nc);
        int32_t P = 0, s0 = 0, s1 = 0, rank = 0;
        uint64_t mk = 0;
        uint32_t mid = 0;
        if (q < n) {
          P = A[q];
          mk = level_key(p, dir, P);
          mid = p.id[P];
          const int32_t g = (int32_t)((int64_t)nc * q / n);
          s0 = gstart(g, n, nc);
          s1 = gstart(g + 1, n, nc);
        }
        for (int32_t r0 = lo; r0 < hi; r0 += BT) {
          __syncthreads();
          if (r0 + t < hi) {
            const int32_t Q = A[r0 + t];
            tk[t] = level_key(p, dir, Q);
            tid[t] = p.id[Q];
          }
          __syncthreads();
          if (q < n) {
            const int32_t a = s0 > r0 ? s0 : r0;
            const int32_t z = s1 < r0 + BT ? s1 : r0 + BT;
            for (int32_t r = a; r < z; ++r) {
              const uint64_t kk = tk[r - r0];
              const uint32_t id = tid[r - r0];
              rank += (kk < mk) | ((kk == mk) & ((id < mid) | ((id == mid) & (r < q))));
            }
          }
        }
        if (q < n) B[s0 + rank] = P;
      }
      __syncthreads();  // B complete before it is read as the next order
      int32_t *tmp = A;
      A = B;
      B = tmp;
      nc = ps.groups[pass];
    }
    for (int32_t b = t; b < nc; b += BT) {
      const int32_t s0 = gstart(b, n, nc), s1 = gstart(b + 1, n, nc);
      double sum = 0.0;
      for (int32_t r = s0; r < s1; ++r) sum += (double)p.psi[A[r]];
      const T mean = (T)(sum / (double)(s1 - s0));
      for (int32_t r = s0; r < s1; ++r) cm[A[r]] = mean;
    }
    __syncthreads();  // before the next element reuses the LDS tiles
  }
}

}  // namespace

bool cond_alloc(CondBuf &b, int32_t ne, int64_t np, size_t tsize, void *(*alloc)(size_t, void *), void *user) {
  b.ne = ne;
  b.np = np;
  size_t scan_bytes = 0;
  hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int32_t *)nullptr, (int32_t *)nullptr, ne + 1);
  b.temp_bytes = scan_bytes > 0 ? scan_bytes : 256;
  const size_t npl = (size_t)(np > 0 ? np : 1);
  b.cnt = (int32_t *)alloc(((size_t)ne + 1) * 4, user);
  b.off = (int32_t *)alloc(((size_t)ne + 1) * 4, user);
  b.cursor = (int32_t *)alloc((size_t)ne * 4, user);
  b.big = (int32_t *)alloc((size_t)ne * 4, user);
  b.nbig = (int32_t *)alloc(256, user);
  b.list = (int32_t *)alloc(npl * 4, user);
  b.list2 = (int32_t *)alloc(npl * 4, user);
  b.cm = alloc(npl * tsize, user);
  b.temp = alloc(b.temp_bytes, user);
  return b.cnt && b.off && b.cursor && b.big && b.nbig && b.list && b.list2 && b.cm && b.temp;
}

template <typename T>
void launch_cond_means(hipStream_t s, const ModelDev &md, const CondBuf &b, PartDev<T> p) {
  const int32_t ne = b.ne;
  const int64_t np = b.np;
  if (np == 0) return;
  const unsigned gp = (unsigned)((np + 255) / 256);
  (void)hipMemsetAsync(b.cnt, 0, ((size_t)ne + 1) * 4, s);
  hipLaunchKernelGGL(k_cond_count, dim3(gp), dim3(256), 0, s, np, ne, p.e, b.cnt);
  size_t tb = b.temp_bytes;
  hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.cnt, b.off, ne + 1, s);
  (void)hipMemsetAsync(b.cursor, 0, (size_t)ne * 4, s);
  (void)hipMemsetAsync(b.nbig, 0, 4, s);
  hipLaunchKernelGGL(k_cond_fill, dim3(gp), dim3(256), 0, s, np, ne, p.e, b.off, b.cursor, b.list);
  hipLaunchKernelGGL(k_cond_wave<T>, dim3((unsigned)ne), dim3(64), 0, s, ne, md, p, b.cnt, b.off, b.list,
                     b.big, b.nbig, (T *)b.cm);
  hipLaunchKernelGGL(k_cond_block<T>, dim3(512), dim3(BT), 0, s, md, p, b.cnt, b.off, b.list, b.list2, b.big,
                     b.nbig, (T *)b.cm);
}

template void launch_cond_means<float>(hipStream_t, const ModelDev &, const CondBuf &, PartDev<float>);
template void launch_cond_means<double>(hipStream_t, const ModelDev &, const CondBuf &, PartDev<double>);

}  // namespace pdfk
