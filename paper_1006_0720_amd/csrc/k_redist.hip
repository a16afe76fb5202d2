// Particle redistribution (App. D, the improved algorithm) on gfx950.
//
// At the start of a step: the elements are ordered by (particle count,
// element number) with a stable radix sort; the k-th element of that order
// with fewer than min_ppe particles receives from the k-th element from the
// top m = min(min_ppe - N_receiver, N_donor - min_ppe) particles, the donor's
// first ones by increasing id, each taking the whole state of a receiver
// resident (residents by increasing id, cycled); an empty receiver gives the
// moving particle a uniform position in the element (Philox sub-stream 3 of
// the particle's step counter) and it keeps the rest of its state.
//
// Kernels: plan (pairs and move counts from the sorted counts), collect (one
// pass over the particles: members of the paired elements into per-pair
// lists), apply (one workgroup per pair: the m smallest ids by repeated block
// minimum reductions, then the copies).  With no critical element every
// kernel after the sort returns at once.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "pdf_solvers.h"
#include "rng.h"

namespace pdfk {

// counts per element as int32 from the count slot of the element sums
__global__ void k_counts_from_sums(int32_t ne, const double *sums, int stride, int32_t *cnt, int32_t *iota) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  cnt[e] = (int32_t)sums[(size_t)e * stride];
  iota[e] = e;
}

// plan: pair k (critical element k of the order) -> receiver, donor, moves
__global__ void k_redist_plan(int32_t ne, int32_t min_ppe, const int32_t *skey, const int32_t *sval,
                              int4 *plan, int32_t *role, int32_t *psize, int32_t *npairs) {
  const int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= ne) return;
  int32_t sz = 0;
  const int32_t kd = ne - 1 - k;
  if (skey[k] < min_ppe && kd > k) {
    const int32_t nc = skey[k], nd = skey[kd];
    int32_t mv = min_ppe - nc;
    if (nd - min_ppe < mv) mv = nd - min_ppe;
    if (mv > 0) {
      const int32_t c = sval[k], d = sval[kd];
      plan[k] = make_int4(c, d, mv, nc);
      role[c] = k;            // receiver of pair k
      role[d] = -(k + 2);     // donor of pair k
      sz = nd + nc;
      atomicMax(npairs, k + 1);
    }
  }
  if (sz == 0) plan[k] = make_int4(-1, -1, 0, 0);
  psize[k] = sz;
}

// collect: every particle of a paired element into its pair's list
// (receiver residents first, then donor particles; order within is arbitrary)
template <typename T>
__global__ void k_redist_collect(int64_t np, const int32_t *pe, const int32_t *role, const int4 *plan,
                                 const int32_t *poff, int32_t *fill_r, int32_t *fill_d, int32_t *list,
                                 const int32_t *npairs) {
  if (*npairs == 0) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int32_t r = role[pe[i]];
  if (r >= 0) {
    const int32_t pos = atomicAdd(&fill_r[r], 1);
    list[poff[r] + pos] = (int32_t)i;
  } else if (r <= -2) {
    const int32_t k = -r - 2;
    const int32_t pos = atomicAdd(&fill_d[k], 1);
    list[poff[k] + plan[k].w + pos] = (int32_t)i;
  }
}

// smallest id greater than `after` (or any when after < 0) among list[0..n):
// block-wide, returns the particle index (or -1)
__device__ int32_t block_next_by_id(const int32_t *list, int32_t n, const uint32_t *id, int64_t after,
                                    uint64_t *red) {
  uint64_t best = ~0ull;
  for (int32_t t = threadIdx.x; t < n; t += blockDim.x) {
    const int32_t i = list[t];
    const uint64_t v = id[i];
    if ((int64_t)v > after) {
      const uint64_t key = (v << 32) | (uint32_t)i;
      best = key < best ? key : best;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(best, off, 64);
    best = o < best ? o : best;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  uint64_t b = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = red[w] < b ? red[w] : b;
  __syncthreads();
  return b == ~0ull ? -1 : (int32_t)(b & 0xFFFFFFFFu);
}

template <typename T>
__global__ __launch_bounds__(256) void k_redist_apply(const KArgs *ka, PartDev<T> p, const int4 *plan,
                                                      const int32_t *poff, const int32_t *list,
                                                      const int32_t *npairs, uint32_t k0, uint32_t k1,
                                                      uint32_t step, unsigned long long *cnt) {
  constexpr int MAXM = 64;
  __shared__ uint64_t red[4];
  __shared__ int32_t donor[MAXM], recv[MAXM];
  const int32_t np_ = *npairs;
  const MeshDev &m = ka->m;
  for (int32_t k = blockIdx.x; k < np_; k += gridDim.x) {
    const int4 pl = plan[k];
    const int32_t c = pl.x, mv = pl.z, nc = pl.w;
    if (mv <= 0) continue;
    const int32_t *rl = list + poff[k];
    const int32_t *dl = rl + nc;
    // the donor's first mv particles and the receiver's residents, by increasing id
    int64_t after = -1;
    for (int q = 0; q < mv; ++q) {
      const int32_t i = block_next_by_id(dl, (int32_t)(poff[k + 1] - poff[k] - nc), p.id, after, red);
      if (threadIdx.x == 0) donor[q] = i;
      after = (int64_t)p.id[i];
    }
    after = -1;
    for (int q = 0; q < nc; ++q) {
      const int32_t i = block_next_by_id(rl, nc, p.id, after, red);
      if (threadIdx.x == 0) recv[q] = i;
      after = (int64_t)p.id[i];
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)mv) {
      const int32_t P = donor[threadIdx.x];
      if (nc > 0) {
        const int32_t Tr = recv[threadIdx.x % nc];
        p.x[P] = p.x[Tr];
        p.y[P] = p.y[Tr];
        p.u[P] = p.u[Tr];
        p.v[P] = p.v[Tr];
        p.w[P] = p.w[Tr];
        p.om[P] = p.om[Tr];
        p.psi[P] = p.psi[Tr];
      } else {
        const u32x4 r = philox10(p.id[P], step, 3u, 0u, k0, k1);
        double r1 = unif_d(r.a), r2 = unif_d(r.b);
        if (r1 + r2 > 1.0) {
          r1 = 1.0 - r1;
          r2 = 1.0 - r2;
        }
        const ElemGeo g = m.geo[c];
        p.x[P] = (T)(g.x[0] + r1 * (g.x[1] - g.x[0]) + r2 * (g.x[2] - g.x[0]));
        p.y[P] = (T)(g.y[0] + r1 * (g.y[1] - g.y[0]) + r2 * (g.y[2] - g.y[0]));
      }
      p.e[P] = c;
    }
    if (threadIdx.x == 0) atomicAdd(&cnt[PDF_CNT_REDIST], (unsigned long long)mv);
    __syncthreads();
  }
}

// ---- buffers and the launch sequence ----
bool redist_alloc(RedistBuf &b, int32_t ne, int64_t np, void *(*alloc)(size_t, void *), void *user) {
  b.ne = ne;
  b.np = np;
  size_t sort_bytes = 0, scan_bytes = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (int32_t *)nullptr, (int32_t *)nullptr,
                                         (int32_t *)nullptr, (int32_t *)nullptr, ne) != hipSuccess ||
      hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int32_t *)nullptr, (int32_t *)nullptr, ne + 1) !=
          hipSuccess)
    return false;
  b.temp_bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
  b.cnt = (int32_t *)alloc((size_t)ne * 4, user);
  b.iota = (int32_t *)alloc((size_t)ne * 4, user);
  b.skey = (int32_t *)alloc((size_t)ne * 4, user);
  b.sval = (int32_t *)alloc((size_t)ne * 4, user);
  b.role = (int32_t *)alloc((size_t)ne * 4, user);
  b.plan = (int4 *)alloc((size_t)ne * sizeof(int4), user);
  b.psize = (int32_t *)alloc(((size_t)ne + 1) * 4, user);
  b.poff = (int32_t *)alloc(((size_t)ne + 1) * 4, user);
  b.fill = (int32_t *)alloc((size_t)ne * 2 * 4, user);
  b.list = (int32_t *)alloc((size_t)(np > 0 ? np : 1) * 4, user);
  b.npairs = (int32_t *)alloc(256, user);
  b.temp = alloc(b.temp_bytes > 0 ? b.temp_bytes : 256, user);
  return b.cnt && b.iota && b.skey && b.sval && b.role && b.plan && b.psize && b.poff && b.fill && b.list &&
         b.npairs && b.temp;
}

template <typename T>
hipError_t launch_redistribute(hipStream_t s, const KArgs *dka, const RedistBuf &b, const double *sums, int stride,
                               PartDev<T> p, int32_t min_ppe, uint64_t seed, uint32_t step,
                               unsigned long long *cnt) {
  const int32_t ne = b.ne;
  const unsigned ge = (unsigned)((ne + 255) / 256);
  hipLaunchKernelGGL(k_counts_from_sums, dim3(ge), dim3(256), 0, s, ne, sums, stride, b.cnt, b.iota);
  size_t tb = b.temp_bytes;
  hipError_t he = hipcub::DeviceRadixSort::SortPairs(b.temp, tb, b.cnt, b.skey, b.iota, b.sval, ne, 0, 32, s);
  if (he != hipSuccess) return he;
  (void)hipMemsetAsync(b.role, 0xFF, (size_t)ne * 4, s);  // -1: no role
  (void)hipMemsetAsync(b.npairs, 0, 4, s);
  (void)hipMemsetAsync(b.psize + ne, 0, 4, s);
  hipLaunchKernelGGL(k_redist_plan, dim3(ge), dim3(256), 0, s, ne, min_ppe, b.skey, b.sval, b.plan, b.role,
                     b.psize, b.npairs);
  tb = b.temp_bytes;
  he = hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.psize, b.poff, ne + 1, s);
  if (he != hipSuccess) return he;
  (void)hipMemsetAsync(b.fill, 0, (size_t)ne * 2 * 4, s);
  hipLaunchKernelGGL(k_redist_collect<T>, dim3((unsigned)((b.np + 255) / 256)), dim3(256), 0, s, b.np, p.e,
                     b.role, b.plan, b.poff, b.fill, b.fill + ne, b.list, b.npairs);
  hipLaunchKernelGGL(k_redist_apply<T>, dim3(1024), dim3(256), 0, s, dka, p, b.plan, b.poff, b.list, b.npairs,
                     (uint32_t)seed, (uint32_t)(seed >> 32), step, cnt);
  return hipGetLastError();
}

template hipError_t launch_redistribute<float>(hipStream_t, const KArgs *, const RedistBuf &, const double *, int,
                                               PartDev<float>, int32_t, uint64_t, uint32_t, unsigned long long *);
template hipError_t launch_redistribute<double>(hipStream_t, const KArgs *, const RedistBuf &, const double *, int,
                                                PartDev<double>, int32_t, uint64_t, uint32_t,
                                                unsigned long long *);

}  // namespace pdfk
