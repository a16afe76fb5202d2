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
// number of group members before it in (key, id) order.  The keys are
// compared as integers (an order-preserving map of the float bits, -0 taken
// as +0); in FP32 the key and the id form one 64-bit word.  Ids are unique,
// so the ranks are a permutation; FP64 and the large-element path also break
// ties of equal ids by position, and the FP32 LDS path pre-fills its target
// positions, so that no input can make an index leave its element.
//
// Launch sequence: count the particles per element (runs merged per wave,
// then an LDS hash table per tile), scan, list the particles of every element
// the same way; one 64-thread workgroup per element with at most 128
// particles, its particles staged in LDS; elements of 129-512 particles the
// same with larger LDS arrays; larger elements go to 256-thread workgroups
// that keep the order in global memory and count ranks over LDS tiles.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "pdf_solvers.h"

namespace pdfk {

namespace {

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

// entry k of a 3-array by selects (a dynamic index would go through scratch)
__device__ __forceinline__ int32_t pick3(const int32_t (&a)[3], int k) { return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]); }

__device__ __forceinline__ Passes plan_passes(const ModelDev &md, int32_t n) {
  const int32_t f[3] = {md.cond_nu, md.cond_nv, md.cond_nw};
  Passes ps;
  ps.n_pass = 0;
  ps.dir[0] = -1;  // with no level taken: one pass by id
  ps.dir[1] = ps.dir[2] = 0;
  ps.groups[0] = 1;
  ps.groups[1] = ps.groups[2] = 1;
  int32_t nc = 1;
  bool go = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!go || f[d] <= 1) continue;
    const int32_t next = nc * f[d];
    if (n / next < md.cond_min) {  // the adaptive stop
      go = false;
      continue;
    }
    // slot ps.n_pass, written through selects (a dynamic index goes through scratch)
    const int k = ps.n_pass;
    if (k == 0) {
      ps.dir[0] = d;
      ps.groups[0] = next;
    } else if (k == 1) {
      ps.dir[1] = d;
      ps.groups[1] = next;
    } else {
      ps.dir[2] = d;
      ps.groups[2] = next;
    }
    ps.n_pass++;
    nc = next;
  }
  if (ps.n_pass == 0) ps.n_pass = 1;
  return ps;
}

__device__ __forceinline__ int32_t gstart(int64_t g, int64_t n, int64_t P) { return (int32_t)((g * n + P - 1) / P); }
// the same in 32 bits for the LDS paths (n <= CAP_M): every level keeps at
// least one particle per group, so P <= n and g * n + P stays below 2^19
__device__ __forceinline__ int32_t gstart32(uint32_t g, uint32_t n, uint32_t P) { return (int32_t)((g * n + P - 1) / P); }
__device__ __forceinline__ int32_t group_of32(uint32_t q, uint32_t n, uint32_t P) { return (int32_t)(P * q / n); }

// barrier of the NT threads that share one element's LDS: a whole workgroup,
// or (NT = 64) one wave, whose LDS accesses complete in issue order
template <int NT>
__device__ __forceinline__ void grp_sync() {
  if constexpr (NT == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

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

// ---- per-element particle lists ------------------------------------------
// A workgroup takes a tile of TT * TP consecutive particles.  Equal elements
// in consecutive lanes are merged first (wave_runs); the run heads then add
// their run lengths into an LDS hash table keyed by element, so that each
// distinct element of the tile costs one global atomic.  A run whose element
// finds no table slot goes to global memory directly.
constexpr int TT = 256, TP = 8;
constexpr int HS_LOG2 = 10, HS = 1 << HS_LOG2;

__device__ __forceinline__ int hslot(int32_t *hk, int32_t e) {
  uint32_t h = ((uint32_t)e * 2654435761u) >> (32 - HS_LOG2);
  for (int probe = 0; probe < 32; ++probe) {
    const int32_t k = __hip_atomic_load(&hk[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (k == e) return (int)h;
    if (k == -1) {
      const int32_t old = atomicCAS(&hk[h], -1, e);
      if (old == -1 || old == e) return (int)h;
    }
    h = (h + 1u) & (uint32_t)(HS - 1);
  }
  return -1;
}

// counts from the count slot of the element sums of the last accumulation
__global__ void k_cond_counts_from_sums(int32_t ne, const double *sums, int32_t *cnt) {
  const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) cnt[e] = (int32_t)sums[(size_t)e * NSUM];
}

__global__ __launch_bounds__(TT) void k_cond_count(int64_t np, int32_t ne, const int32_t *pe, int32_t *cnt) {
  __shared__ int32_t hk[HS], hc[HS];
  const int t = threadIdx.x, lane = t & 63;
  for (int s = t; s < HS; s += TT) {
    hk[s] = -1;
    hc[s] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TT * TP;
  int32_t pe_[TP];  // every element number loaded before the first atomic
#pragma unroll
  for (int j = 0; j < TP; ++j) {
    const int64_t i = base + (int64_t)j * TT + t;
    pe_[j] = i < np ? pe[i] : -1;
  }
  for (int j = 0; j < TP; ++j) {
    const int32_t e = pe_[j];
    const bool valid = e >= 0 && e < ne;
    int hl, len;
    wave_runs(e, valid, hl, len);
    if (hl == lane) {
      const int s = hslot(hk, e);
      if (s >= 0)
        atomicAdd(&hc[s], len);
      else
        atomicAdd(&cnt[e], len);
    }
  }
  __syncthreads();
  for (int s = t; s < HS; s += TT) {
    const int32_t k = hk[s];
    if (k >= 0) atomicAdd(&cnt[k], hc[s]);
  }
}

__global__ __launch_bounds__(TT) void k_cond_fill(int64_t np, int32_t ne, const int32_t *pe, const int32_t *off,
                                                  int32_t *cursor, int32_t *list) {
  __shared__ int32_t hk[HS], hc[HS], hb[HS];
  const int t = threadIdx.x, lane = t & 63;
  for (int s = t; s < HS; s += TT) {
    hk[s] = -1;
    hc[s] = 0;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TT * TP;
  int32_t pe_[TP], slot[TP], rank[TP];
  // every element number loaded before the first atomic, so that the loads
  // overlap instead of waiting one by one, and the elements' offsets right
  // after them, in flight during the ranking
#pragma unroll
  for (int j = 0; j < TP; ++j) {
    const int64_t i = base + (int64_t)j * TT + t;
    pe_[j] = i < np ? pe[i] : -1;
  }
  int32_t o0[TP], o1[TP];
#pragma unroll
  for (int j = 0; j < TP; ++j) {
    const int32_t ec = pe_[j] >= 0 && pe_[j] < ne ? pe_[j] : 0;  // unconditional loads, in bounds
    o0[j] = off[ec];
    o1[j] = off[ec + 1];
  }
#pragma unroll
  for (int j = 0; j < TP; ++j) {
    const int32_t e = pe_[j];
    const bool valid = e >= 0 && e < ne;
    int hl, len;
    wave_runs(e, valid, hl, len);
    int s = -1, r = 0;
    if (hl == lane) {
      s = hslot(hk, e);
      r = s >= 0 ? atomicAdd(&hc[s], len) : atomicAdd(&cursor[e], len);  // no slot: the global base
    }
    const int src = hl < 0 ? lane : hl;
    s = __shfl(s, src, 64);
    r = __shfl(r, src, 64) + (lane - src);
    pe_[j] = valid ? e : -1;
    slot[j] = s;
    rank[j] = r;
  }
  __syncthreads();
  for (int s = t; s < HS; s += TT) {
    const int32_t k = hk[s];
    if (k >= 0) hb[s] = atomicAdd(&cursor[k], hc[s]);
  }
  __syncthreads();
  // every destination before the first store (a store between the loads and
  // their use makes the compiler wait for all memory operations)
  int32_t dst[TP];
#pragma unroll
  for (int j = 0; j < TP; ++j) {
    dst[j] = -1;
    if (pe_[j] < 0) continue;
    const int32_t pos = slot[j] >= 0 ? hb[slot[j]] + rank[j] : rank[j];
    if (pos < o1[j] - o0[j]) dst[j] = o0[j] + pos;  // counts that disagree with the elements stay in bounds
  }
  __builtin_amdgcn_sched_barrier(0);  // keeps the stores after every destination
#pragma unroll
  for (int j = 0; j < TP; ++j)
    if (dst[j] >= 0) list[dst[j]] = (int32_t)(base + (int64_t)j * TT + t);
}

// ---- sort and divide in LDS: one element of at most CAP particles per
// 64-thread workgroup ----
constexpr int CAP_S = 128, CAP_M = 512;
// elements per wave of k_cond_small: with 1 to 4 the step times agree within
// 1.5 % at 100M particles, 2 the fastest; longer runs per wave leave a long
// last round of workgroups (the chip holds about 1800 at once) and lose
constexpr int32_t SMALL_PER_WAVE = 2;

template <typename T, int CAP>
struct CondLds {
  // by slot (the element's list order); the U keys' space also holds the
  // bucket counts and starts of the first division by buckets
  union {
    T ku[CAP];
    int32_t kh[CAP * sizeof(T) / 4];
  };
  T kv[CAP], kw[CAP], psi[CAP];
  uint32_t id[CAP];
  int32_t idx[CAP];
  // by position: the sort key (FP32: the 32-bit key over the id in one word;
  // FP64: the 64-bit key, the id apart) and the slot, rewritten in place by
  // every pass once all of its ranks are counted
  uint64_t k[CAP];
  uint32_t ki[sizeof(T) == 8 ? CAP : 1];
  uint16_t s[CAP];
};

template <typename T, int CAP>
__device__ __forceinline__ void set_key(CondLds<T, CAP> &L, int pos, int slot, int dir) {
  if constexpr (sizeof(T) == 4) {
    const uint64_t kk = dir < 0 ? 0 : ordkey(dir == 0 ? L.ku[slot] : (dir == 1 ? L.kv[slot] : L.kw[slot]));
    L.k[pos] = (kk << 32) | L.id[slot];
  } else {
    L.k[pos] = dir < 0 ? 0 : ordkey(dir == 0 ? L.ku[slot] : (dir == 1 ? L.kv[slot] : L.kw[slot]));
    L.ki[pos] = L.id[slot];
  }
}

// rank of position q within its group [s0, s1) in (key, id, position) order
template <typename T, int CAP>
__device__ __forceinline__ int32_t rank_in(const CondLds<T, CAP> &L, int32_t s0, int32_t s1, int32_t q) {
  const uint64_t mk = L.k[q];
  int32_t rank = 0;
  if constexpr (sizeof(T) == 4) {
    // (key, id) in one word, unique while the ids are
#pragma unroll 8
    for (int32_t r = s0; r < s1; ++r) rank += L.k[r] < mk;
  } else {
    const uint32_t mi = L.ki[q];
#pragma unroll 8
    for (int32_t r = s0; r < s1; ++r) {
      const uint64_t k = L.k[r];
      const uint32_t id = L.ki[r];
      rank += (k < mk) | ((k == mk) & ((id < mi) | ((id == mi) & (r < q))));
    }
  }
  return rank;
}

// FP32 rank of key mk within the group [s0, s0 + len), where every group of the
// division has lmin (uniform over the threads) or lmin + 1 members: the first
// lmin members in a loop the threads share, the possible extra one after it
template <int CAP>
__device__ __forceinline__ int32_t rank_in_even(const CondLds<float, CAP> &L, int32_t s0, int32_t len, int32_t lmin,
                                                uint64_t mk) {
  const uint64_t *kp = L.k + s0;
  int32_t rank = 0;
#pragma unroll 4
  for (int32_t r = 0; r < lmin; ++r) rank += kp[r] < mk;
  if (len > lmin) rank += kp[lmin] < mk;
  return rank;
}

// the first division (one group): each thread ranks its QP positions in one
// sweep over all n keys, read once per sweep (QP * NT >= n)
template <typename T, int CAP, int NT, int QP>
__device__ __forceinline__ void rank_all(const CondLds<T, CAP> &L, int32_t n, int32_t rank[], int t) {
  uint64_t mk[QP];
  uint32_t mi[QP];
#pragma unroll
  for (int j = 0; j < QP; ++j) {
    const int32_t q = t + j * NT;
    mk[j] = q < n ? L.k[q] : 0;
    if constexpr (sizeof(T) == 8) mi[j] = q < n ? L.ki[q] : 0;
    rank[j] = 0;
  }
#pragma unroll 4
  for (int32_t r = 0; r < n; ++r) {
    const uint64_t k = L.k[r];
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int j = 0; j < QP; ++j) rank[j] += k < mk[j];
    } else {
      const uint32_t id = L.ki[r];
#pragma unroll
      for (int j = 0; j < QP; ++j)
        rank[j] += (k < mk[j]) | ((k == mk[j]) & ((id < mi[j]) | ((id == mi[j]) & (r < t + j * NT))));
    }
  }
}

// the first division by velocity buckets (FP32, one wave per element, first
// level by U): a map that never decreases with U spreads the keys over NB
// buckets, so every key of a lower bucket is smaller and equal velocities share
// a bucket; a position's rank is the start of its bucket plus its rank among
// that bucket's keys, the same (key, id) rank as the full sweep.  Returns false
// with LDS untouched, for the full sweep, when a velocity is not finite.
constexpr int NB = 64;
template <int CAP>
__device__ __forceinline__ bool rank_buckets(CondLds<float, CAP> &L, int32_t n, int32_t rank[], int lane) {
  constexpr int QP = CAP / 64;
  static_assert(CAP >= 2 * NB, "the bucket counts and starts fit the U keys' space");
  float u[QP];
  uint64_t mk[QP];
  float lo = INFINITY, hi = -INFINITY;
  bool bad = false;
#pragma unroll
  for (int j = 0; j < QP; ++j) {
    const int32_t q = lane + j * 64;
    u[j] = 0.0f;
    mk[j] = 0;
    if (q < n) {
      u[j] = L.ku[q];  // the first pass still has the list order
      mk[j] = L.k[q];
      bad |= !__builtin_isfinite(u[j]);
      lo = fminf(lo, u[j]);
      hi = fmaxf(hi, u[j]);
    }
  }
  if (__ballot(bad) != 0) return false;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, m, 64));
    hi = fmaxf(hi, __shfl_xor(hi, m, 64));
  }
  // zero spread, or one too narrow or too wide for a finite scale: one bucket
  float scale = (float)NB / (hi - lo);
  if (!(scale <= __FLT_MAX__)) scale = 0.0f;
  int32_t *cnt = L.kh, *start = L.kh + NB;
  grp_sync<64>();  // every lane holds its U values before their space is reused
  cnt[lane] = 0;
  grp_sync<64>();
  int32_t b[QP], c[QP];
#pragma unroll
  for (int j = 0; j < QP; ++j) {
    b[j] = 0;
    c[j] = 0;
    if (lane + j * 64 < n) {
      // (u - lo) and the product are correctly rounded, so they never decrease with u
      const int32_t bb = scale > 0.0f ? (int32_t)((u[j] - lo) * scale) : 0;
      b[j] = bb < NB - 1 ? bb : NB - 1;
      c[j] = atomicAdd(&cnt[b[j]], 1);
    }
  }
  grp_sync<64>();
  const int32_t mine = cnt[lane];
  int32_t incl = mine;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const int32_t o = __shfl_up(incl, m, 64);
    if (lane >= m) incl += o;
  }
  start[lane] = incl - mine;
  grp_sync<64>();
  // the keys in bucket order over the sweep's key array, then the ranks
#pragma unroll
  for (int j = 0; j < QP; ++j)
    if (lane + j * 64 < n) L.k[start[b[j]] + c[j]] = mk[j];
  grp_sync<64>();
#pragma unroll
  for (int j = 0; j < QP; ++j) {
    rank[j] = 0;
    if (lane + j * 64 < n) {
      const int32_t s0 = start[b[j]], s1 = s0 + cnt[b[j]];
      int32_t r = 0;
      for (int32_t k = s0; k < s1; ++k) r += L.k[k] < mk[j];
      rank[j] = s0 + r;
    }
  }
  return true;
}

// one element's particles as a thread holds them between their loads and LDS
template <typename T, int QP>
struct Held {
  int32_t gi[QP];  // particle indices (the list entries)
  uint32_t id[QP];
  T u[QP], v[QP], w[QP], psi[QP];
};

// the list entries of the n > 0 particles of an element (list[base, base+n)).
// Every load is unconditional, a thread past the end reading the last entry
// again: loads under a per-thread branch would each wait for the ones before
template <typename T, int QP, int NT>
__device__ __forceinline__ void load_list(Held<T, QP> &h, const int32_t *list, int32_t base, int32_t n, int t) {
#pragma unroll
  for (int j = 0; j < QP; ++j) {
    const int32_t q = t + j * NT;
    h.gi[j] = list[base + (q < n ? q : n - 1)];
  }
}

// the particles of the list entries held (after load_list with n > 0)
template <typename T, int QP, int NT>
__device__ __forceinline__ void load_particles(Held<T, QP> &h, const PartDev<T> &p) {
#pragma unroll
  for (int j = 0; j < QP; ++j) {
    const int32_t i = h.gi[j];
    h.id[j] = p.id[i];
    h.u[j] = p.u[i];
    h.v[j] = p.v[i];
    h.w[j] = p.w[i];
    h.psi[j] = p.psi[i];
  }
}

template <typename T, int CAP, int QP, int NT>
__device__ __forceinline__ void store_held(CondLds<T, CAP> &L, const Held<T, QP> &h, int32_t n, int t) {
#pragma unroll
  for (int j = 0; j < QP; ++j) {
    const int32_t q = t + j * NT;
    if (q >= n) continue;
    L.idx[q] = h.gi[j];
    L.id[q] = h.id[j];
    L.ku[q] = h.u[j];
    L.kv[q] = h.v[j];
    L.kw[q] = h.w[j];
    L.psi[q] = h.psi[j];
  }
}

// sort and divide the n <= CAP particles of one element, staged in LDS by
// store_held, with NT threads (t = 0..NT-1), and write every particle's bin mean
template <typename T, int CAP, int NT>
__device__ void cond_solve(CondLds<T, CAP> &L, const ModelDev &md, int32_t n, T *cm, int t) {
  constexpr int QP = CAP / NT;
  grp_sync<NT>();
  const Passes ps = plan_passes(md, n);
  for (int q = t; q < n; q += NT) {
    L.s[q] = (uint16_t)q;
    set_key(L, q, q, ps.dir[0]);
  }
  grp_sync<NT>();
  int32_t nc = 1;
  for (int pass = 0; pass < ps.n_pass; ++pass) {
    const bool more = pass + 1 < ps.n_pass;
    const int nextdir = more ? pick3(ps.dir, pass + 1) : 0;
    // FP32 ranks are strict-order counts, a permutation only while the ids are
    // unique; a rank stays below the end of its group, and a position that no
    // rank hits keeps its slot of the last pass, so repeated ids can only give
    // wrong bins, never an index outside the element
    int32_t rank[QP];
    bool ranked = false;
    if constexpr (sizeof(T) == 4 && NT == 64) {
      if (nc == 1 && ps.dir[0] == 0) ranked = rank_buckets<CAP>(L, n, rank, t);
    }
    if (!ranked && nc == 1) {
      // one position per thread when the element allows (n is uniform over the
      // threads of the element)
      if (QP > 1 && n <= NT) {
        rank_all<T, CAP, NT, 1>(L, n, rank, t);
#pragma unroll
        for (int j = 1; j < QP; ++j) rank[j] = 0;
      } else {
        rank_all<T, CAP, NT, QP>(L, n, rank, t);
      }
    } else if (!ranked) {
      const int32_t lmin = n / nc;  // the groups hold lmin or lmin + 1 members
#pragma unroll
      for (int j = 0; j < QP; ++j) {
        const int32_t q = t + j * NT;
        rank[j] = 0;
        if (q < n) {
          const int32_t g = group_of32(q, n, nc);
          const int32_t s0 = gstart32(g, n, nc), s1 = gstart32(g + 1, n, nc);
          if constexpr (sizeof(T) == 4)
            rank[j] = s0 + rank_in_even(L, s0, s1 - s0, lmin, L.k[q]);
          else
            rank[j] = s0 + rank_in(L, s0, s1, q);
        }
      }
    }
    // every rank is counted and every slot read before the order is rewritten
    int sl[QP];
#pragma unroll
    for (int j = 0; j < QP; ++j) {
      const int32_t q = t + j * NT;
      sl[j] = q < n ? L.s[q] : 0;
    }
    grp_sync<NT>();
#pragma unroll
    for (int j = 0; j < QP; ++j) {
      const int32_t q = t + j * NT;
      if (q < n) {
        const int np_ = rank[j];  // the group start is 0 for the single group
        L.s[np_] = (uint16_t)sl[j];
        if (more) set_key(L, np_, sl[j], nextdir);
      }
    }
    grp_sync<NT>();
    nc = pick3(ps.groups, pass);
  }
  // bin means (App. B), each bin summed in the order of its positions
  for (int32_t b = t; b < nc; b += NT) {
    const int32_t s0 = gstart32(b, n, nc), s1 = gstart32(b + 1, n, nc);
    double sum = 0.0;
    for (int32_t r = s0; r < s1; ++r) sum += (double)L.psi[L.s[r]];
    const T mean = (T)(sum / (double)(s1 - s0));
    for (int32_t r = s0; r < s1; ++r) cm[L.idx[L.s[r]]] = mean;
  }
}

// one element from its list: every list entry of the thread first, then every
// particle load, so that the gather waits on two rounds of global loads
template <typename T, int CAP, int NT>
__device__ void cond_element(CondLds<T, CAP> &L, const ModelDev &md, const PartDev<T> &p, int32_t n, int32_t base,
                             const int32_t *list, T *cm, int t) {
  constexpr int QP = CAP / NT;
  if (n <= 0) return;
  Held<T, QP> h;
  load_list<T, QP, NT>(h, list, base, n, t);
  load_particles<T, QP, NT>(h, p);
  store_held<T, CAP, QP, NT>(L, h, n, t);
  cond_solve<T, CAP, NT>(L, md, n, cm, t);
}

// every element: those of at most CAP_S particles here, one per wave at a
// time (SW waves per workgroup, each with its own LDS), the others listed for
// the mid-size and large-element kernels
constexpr int SW = 4;
template <typename T>
__global__ __launch_bounds__(64 * SW) void k_cond_small(int32_t ne, ModelDev md, PartDev<T> p, const int32_t *cnt,
                                                        const int32_t *off, const int32_t *list, int32_t *mid,
                                                        int32_t *big, int32_t *counters, T *cm) {
  __shared__ CondLds<T, CAP_S> L[SW];
  // the wave number through readfirstlane: it makes the element and all that
  // follows from it (counts, group bounds, loop trips) wave-uniform to the
  // compiler, which then keeps them in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  constexpr int QP = CAP_S / 64;
  const int64_t stride = (int64_t)gridDim.x * SW;
  // a software pipeline over the wave's elements e, e + stride, ...: the
  // particle loads of one element go out together with the list entries of
  // the next and the counts of the one after, so that each element waits on
  // one round of global loads
  auto counts = [&](int64_t x, int32_t &nx, int32_t &fx) {
    nx = 0;
    fx = 0;
    if (x < ne) {
      nx = cnt[x];
      fx = off[x];
    }
  };
  int64_t e = (int64_t)blockIdx.x * SW + w;
  int32_t n, first, n1, first1;
  counts(e, n, first);
  counts(e + stride, n1, first1);
  Held<T, QP> h;
  if (n > 0 && n <= CAP_S) load_list<T, QP, 64>(h, list, first, n, lane);
  while (e < ne) {
    const int32_t m = n <= CAP_S ? n : 0;  // the particles sorted here
    if (m > 0) load_particles<T, QP, 64>(h, p);
    Held<T, QP> h1;
    if (n1 > 0 && n1 <= CAP_S) load_list<T, QP, 64>(h1, list, first1, n1, lane);
    int32_t n2, first2;
    counts(e + 2 * stride, n2, first2);
    if (n > CAP_S && lane == 0) {
      if (n > CAP_M)
        big[atomicAdd(&counters[0], 1)] = (int32_t)e;
      else
        mid[atomicAdd(&counters[1], 1)] = (int32_t)e;
    }
    if (m > 0) {
      store_held<T, CAP_S, QP, 64>(L[w], h, m, lane);
      cond_solve<T, CAP_S, 64>(L[w], md, m, cm, lane);
      grp_sync<64>();  // before the wave's next element overwrites its LDS
    }
    e += stride;
    n = n1;
    first = first1;
    n1 = n2;
    first1 = first2;
#pragma unroll
    for (int j = 0; j < QP; ++j) h.gi[j] = h1.gi[j];
  }
}

// the listed elements of CAP_S+1..CAP_M particles, one per 256-thread
// workgroup (the grid covers every element; workgroups beyond the list exit)
template <typename T>
__global__ __launch_bounds__(256) void k_cond_mid(ModelDev md, PartDev<T> p, const int32_t *cnt, const int32_t *off,
                                                  const int32_t *list, const int32_t *mid, const int32_t *counters,
                                                  T *cm) {
  __shared__ CondLds<T, CAP_M> L;
  const int32_t nm = counters[1];
  for (int32_t k = blockIdx.x; k < nm; k += gridDim.x) {
    const int32_t e = mid[k];
    cond_element<T, CAP_M, 256>(L, md, p, cnt[e], off[e], list, cm, threadIdx.x);
    __syncthreads();  // before the next element overwrites the LDS
  }
}

// elements of more than CAP_M particles: one 256-thread workgroup each, the
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
      const int dir = pick3(ps.dir, pass);
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
      nc = pick3(ps.groups, pass);
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
  if (hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int32_t *)nullptr, (int32_t *)nullptr, ne + 1) !=
      hipSuccess)
    return false;
  b.temp_bytes = scan_bytes > 0 ? scan_bytes : 256;
  const size_t npl = (size_t)(np > 0 ? np : 1);
  b.cnt = (int32_t *)alloc(((size_t)ne + 1) * 4, user);
  b.off = (int32_t *)alloc(((size_t)ne + 1) * 4, user);
  b.cursor = (int32_t *)alloc((size_t)ne * 4, user);
  b.big = (int32_t *)alloc((size_t)ne * 4, user);
  b.mid = (int32_t *)alloc((size_t)ne * 4, user);
  b.nbig = (int32_t *)alloc(256, user);  // [0] large elements listed, [1] mid-size
  b.list = (int32_t *)alloc(npl * 4, user);
  b.list2 = (int32_t *)alloc(npl * 4, user);
  b.cm = alloc(npl * tsize, user);
  b.temp = alloc(b.temp_bytes, user);
  return b.cnt && b.off && b.cursor && b.big && b.mid && b.nbig && b.list && b.list2 && b.cm && b.temp;
}

template <typename T>
hipError_t launch_cond_means(hipStream_t s, const ModelDev &md, const CondBuf &b, PartDev<T> p,
                             const double *elem_sums) {
  const int32_t ne = b.ne;
  const int64_t np = b.np;
  if (np == 0) return hipSuccess;
  const unsigned gt = (unsigned)((np + (int64_t)TT * TP - 1) / ((int64_t)TT * TP));
  (void)hipMemsetAsync(b.cnt, 0, ((size_t)ne + 1) * 4, s);
  if (elem_sums)
    hipLaunchKernelGGL(k_cond_counts_from_sums, dim3((ne + 255) / 256), dim3(256), 0, s, ne, elem_sums, b.cnt);
  else
    hipLaunchKernelGGL(k_cond_count, dim3(gt), dim3(TT), 0, s, np, ne, p.e, b.cnt);
  size_t tb = b.temp_bytes;
  const hipError_t se = hipcub::DeviceScan::ExclusiveSum(b.temp, tb, b.cnt, b.off, ne + 1, s);
  if (se != hipSuccess) return se;
  (void)hipMemsetAsync(b.cursor, 0, (size_t)ne * 4, s);
  (void)hipMemsetAsync(b.nbig, 0, 8, s);
  hipLaunchKernelGGL(k_cond_fill, dim3(gt), dim3(TT), 0, s, np, ne, p.e, b.off, b.cursor, b.list);
  T *cm = (T *)b.cm;
  const int32_t gs = (int32_t)(((int64_t)ne + SW * SMALL_PER_WAVE - 1) / (SW * SMALL_PER_WAVE));
  hipLaunchKernelGGL(k_cond_small<T>, dim3((unsigned)gs), dim3(64 * SW), 0, s, ne,
                     md, p, b.cnt, b.off, b.list, b.mid, b.big, b.nbig, cm);
  hipLaunchKernelGGL(k_cond_mid<T>, dim3((unsigned)(ne < 65536 ? ne : 65536)), dim3(256), 0, s, md, p, b.cnt, b.off,
                     b.list, b.mid, b.nbig, cm);
  hipLaunchKernelGGL(k_cond_block<T>, dim3(512), dim3(BT), 0, s, md, p, b.cnt, b.off, b.list, b.list2, b.big,
                     b.nbig, cm);
  return hipGetLastError();
}

template hipError_t launch_cond_means<float>(hipStream_t, const ModelDev &, const CondBuf &, PartDev<float>,
                                       const double *);
template hipError_t launch_cond_means<double>(hipStream_t, const ModelDev &, const CondBuf &, PartDev<double>,
                                        const double *);

}  // namespace pdfk
