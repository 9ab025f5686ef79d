// gfx950 block-Jacobi preconditioned conjugate gradients on the reduced
// camera system: one cooperative launch per solve.
//
// Layout (HBM): upper blocks S[e][81] of the reduced camera matrix (T),
// diagonal blocks Sdiag[a][81] and block-Jacobi factors Minv[a][81] (FP64),
// right-hand side b and solution x [n_cams][9] (FP64); exchange rings zring,
// partA, partB of (maxiter + 1) write-once slots.
#include "ba_device.h"
#include "ba_internal.h"
#include "ba_kernels.h"
#include "ba_reduce.h"

namespace ba {

// ---------------------------------------------------------------------------
// block-Jacobi preconditioned conjugate gradients on S x = bS (Sec. IV-C-2),
// one cooperative launch for the whole solve (the paper removes per-iteration
// launch overhead by replaying a captured PCG iteration, App. B; here the
// iterations never leave the GPU).
//
// Workgroup B owns the contiguous block rows [wg_row[B], wg_row[B+1]), chosen
// on the host so that workgroups hold similar numbers of (row, block) items.
// Its own-row vectors and block-Jacobi factors stay in LDS for the whole
// solve.  The items are split into SPMV_GROUPS contiguous ranges; 9 lanes
// share an item, lane `comp` holding row `comp` of the block (column `comp`
// for a transposed upper block).  When every range has at most PCG_IPG items
// (RES = true) the lanes keep their block values in registers for the whole
// solve; otherwise they are streamed in batches of PCG_IPG each iteration.
//
// Values other workgroups read (the preconditioned residual z, by column,
// and the dot-product partials) are written once per iteration into a fresh
// ring slot with agent-scope (write-through) stores and read after a barrier
// with ordinary cached loads, so iterations need no cache flush.  Dots are
// reduced from the per-workgroup partials in a fixed order, identically in
// every workgroup, so every workgroup takes the same branch.  Standard PCG
// recurrence; the product S p_k is formed as S z_k + beta q_{k-1}, so the
// direction update and the product share one barrier (two per iteration).
// ---------------------------------------------------------------------------
constexpr int SPMV_GROUPS = PCG_THREADS / 9;

// Workgroup b of the grid runs on XCD b % 8 (round-robin dispatch); it takes
// the row range of index xcd_block(b): each XCD gets a contiguous run of row
// ranges, so the z columns a workgroup reads come mostly from workgroups of
// its own XCD, whose write-through stores leave the lines in that XCD's L2.
// A bijection of [0, G).
__device__ __forceinline__ int xcd_block(int b, int G) {
  const int x = b & 7, n8 = G >> 3, rem = G & 7;
  return x * n8 + min(x, rem) + (b >> 3);
}
// A workgroup-uniform FP64 value held in scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// 64-bit DPP move; rows outside ROWS, and lanes the control gives no
// source, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_mov(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// Sum over a full wavefront in a fixed order through DPP lane moves (no
// LDS traffic): quads, rows of 16, then rows 1 and 3 take rows 0 and 2,
// rows 2 and 3 take lane 31.  The total is valid in lane 63.
__device__ __forceinline__ double dpp_wave_total(double v) {
  v += dpp_mov<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x124, 0xF>(v);  // row_ror:4
  v += dpp_mov<0x128, 0xF>(v);  // row_ror:8
  v += dpp_mov<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_mov<0x143, 0xC>(v);  // row_bcast:31
  return v;
}

constexpr long BARRIER_SPIN_LIMIT = 1L << 21;

__device__ __forceinline__ void publish(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned agent_add(unsigned* p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void agent_store(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier of a co-resident grid without cache flushes: every wave
// waits for its own memory operations to complete, one thread per workgroup
// arrives on its group's counter (BARRIER_FANIN workgroups per group), the
// last of a group arrives on the top counter, and the last overall advances
// the generation the others poll.  The wait is bounded: on timeout the sticky
// error flag is raised, and once it is set every later barrier returns at
// once, so the kernel always terminates.
__device__ __forceinline__ bool grid_barrier(GridSync* gs, int* error) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  __shared__ int failed;
  if (threadIdx.x == 0) {
    int f = __hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER;
    if (!f && gridDim.x > 1) {
      const unsigned gen = __hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned grp = blockIdx.x / BARRIER_FANIN;
      const unsigned ngrp = (gridDim.x + BARRIER_FANIN - 1) / BARRIER_FANIN;
      const unsigned gsz = min((unsigned)BARRIER_FANIN, gridDim.x - grp * BARRIER_FANIN);
      bool last = false;
      if (agent_add(&gs->group[grp].count, 1u) == gsz - 1) {
        agent_store(&gs->group[grp].count, 0u);
        __builtin_amdgcn_s_waitcnt(0);
        if (agent_add(&gs->count, 1u) == ngrp - 1) {
          agent_store(&gs->count, 0u);
          __builtin_amdgcn_s_waitcnt(0);
          agent_add(&gs->gen, 1u);
          last = true;
        }
      }
      if (!last) {
        long spins = 0;
        while (__hip_atomic_load(&gs->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          if (++spins > BARRIER_SPIN_LIMIT ||
              (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER)) {
            atomicOr(error, (int)ERR_BARRIER);
            f = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    failed = f;
  }
  __syncthreads();
  return failed == 0;
}

// The pipelined PCG synchronises through the dot-product records themselves:
// before the first barrier every workgroup fills its records of all
// iteration slots with a NaN pattern that arithmetic never produces; in
// iteration i a workgroup publishes its three partials only after its m
// columns have reached memory, and the readers poll the records until no
// word holds the pattern.  One memory round trip replaces the barrier's
// atomics and the separate read of the partials.  Bounded like the
// barrier: on timeout the sticky error flag is raised.
constexpr unsigned long long PCG_PENDING = 0x7FF4DEADBEEF0000ull;

__device__ __forceinline__ void clear_record(double* p) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), PCG_PENDING, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// Thread t < G waits for workgroup t's three partials of slot `rec`; returns
// false on timeout (error flag raised).
__device__ __forceinline__ bool poll_record(const double* rec, double& v0, double& v1, double& v2,
                                            int* error) {
  const unsigned long long* r = reinterpret_cast<const unsigned long long*>(rec);
  long spins = 0;
  while (true) {
    const unsigned long long a0 = __hip_atomic_load(r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long a1 = __hip_atomic_load(r + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long a2 = __hip_atomic_load(r + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a0 != PCG_PENDING && a1 != PCG_PENDING && a2 != PCG_PENDING) {
      v0 = __longlong_as_double((long long)a0);
      v1 = __longlong_as_double((long long)a1);
      v2 = __longlong_as_double((long long)a2);
      return true;
    }
    if (++spins > BARRIER_SPIN_LIMIT ||
        (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER)) {
      atomicOr(error, (int)ERR_BARRIER);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// The register-resident pipelined PCG also marks its own z columns of every
// ring slot after the first pending, so that a reader polls the column words
// it needs together with the dot records, in one round trip: no wait for the
// columns' stores before the partials are published, no separate fetch after
// the poll.  A thread polls PCG_POLL_WORDS column words at a time (one round
// for up to PCG_POLL_WORDS * 1024 / 9 columns, more rounds beyond).
constexpr int PCG_POLL_WORDS = 2;

// Polls the block columns cols[0 .. n) of ring slot zk into LDS zl and, when
// rec is not null, the three words of record rec into v0..v2 (with the first
// round of columns); the loads of all still-pending words of a round are
// issued together.  Returns false on timeout (error flag raised).
__device__ __forceinline__ bool poll_slot(const int32_t* cols, int n, const double* zk, double* zl,
                                          const double* rec, double& v0, double& v1, double& v2,
                                          int* error) {
  const unsigned long long* z = reinterpret_cast<const unsigned long long*>(zk);
  const unsigned long long* r = reinterpret_cast<const unsigned long long*>(rec);
  const int nw = n * 9, tid = threadIdx.x, nt = blockDim.x;
  unsigned want = rec ? 7u << 8 : 0u;  // bit k < PCG_POLL_WORDS: word base + tid + k nt; bits 8..10: rec
  long spins = 0;
  for (int base = 0; base == 0 || base < nw; base += PCG_POLL_WORDS * nt) {
#pragma unroll
    for (int k = 0; k < PCG_POLL_WORDS; ++k)
      if (base + tid + k * nt < nw) want |= 1u << k;
    while (want) {
      unsigned long long w[PCG_POLL_WORDS], rv[3];
#pragma unroll
      for (int k = 0; k < PCG_POLL_WORDS; ++k) {
        w[k] = PCG_PENDING;
        if ((want >> k) & 1u) {
          const int u = base + tid + k * nt, j = u / 9;
          // byte offset below 2^32 (fewer than 2^25 cameras): base + 32-bit offset addressing
          const unsigned boff = ((unsigned)cols[j] * ZSTRIDE + (unsigned)(u - 9 * j)) * 8u;
          w[k] = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(
                                       reinterpret_cast<const char*>(z) + boff),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
#pragma unroll
      for (int q = 0; q < 3; ++q)
        rv[q] = (want >> 8) & 1u ? __hip_atomic_load(r + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                 : PCG_PENDING;
#pragma unroll
      for (int k = 0; k < PCG_POLL_WORDS; ++k)
        if (((want >> k) & 1u) && w[k] != PCG_PENDING) {
          zl[base + tid + k * nt] = __longlong_as_double((long long)w[k]);
          want &= ~(1u << k);
        }
      if (((want >> 8) & 1u) && rv[0] != PCG_PENDING && rv[1] != PCG_PENDING && rv[2] != PCG_PENDING) {
        v0 = __longlong_as_double((long long)rv[0]);
        v1 = __longlong_as_double((long long)rv[1]);
        v2 = __longlong_as_double((long long)rv[2]);
        want = 0u | (want & ((1u << PCG_POLL_WORDS) - 1u));
      }
      if (!want) break;
      if (++spins > BARRIER_SPIN_LIMIT ||
          (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER)) {
        atomicOr(error, (int)ERR_BARRIER);
        return false;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return true;
}

// Block values of a lane group's items (row `comp` of each block, or column
// `comp` of a transposed upper block), with the item's LDS column slot and
// local row.
struct PcgItems {
  double v[PCG_IPG][9];
  int lc[PCG_IPG], rl[PCG_IPG];
};

template <typename T>
__device__ __forceinline__ void pcg_load_items(const PcgArgs& a, int ib, int k0, int k1, const int* rptr,
                                               int comp, PcgItems& it) {
  const T* __restrict__ S = reinterpret_cast<const T*>(a.S);
  int row = 0;
  while (rptr[row + 1] <= k0) ++row;
#pragma unroll
  for (int kk = 0; kk < PCG_IPG; ++kk) {
    const int i = k0 + kk;
    if (i < k1) {
      while (rptr[row + 1] <= i) ++row;
      const int code = a.item_code[ib + i];
      const int e = a.item_e[ib + i];
      it.lc[kk] = code & 0xFFFF;
      it.rl[kk] = row;
      if (code & ITEM_DIAG) {
        const double* Bp = a.Sdiag + (size_t)e * 81 + comp * 9;
#pragma unroll
        for (int m = 0; m < 9; ++m) it.v[kk][m] = Bp[m];
      } else if (code & ITEM_TRANS) {
        const T* Bp = S + (size_t)e * 81 + comp;
#pragma unroll
        for (int m = 0; m < 9; ++m) it.v[kk][m] = (double)Bp[9 * m];
      } else {
        const T* Bp = S + (size_t)e * 81 + comp * 9;
#pragma unroll
        for (int m = 0; m < 9; ++m) it.v[kk][m] = (double)Bp[m];
      }
    } else {
      it.lc[kk] = 0;
      it.rl[kk] = -1;
    }
  }
}

// y[own rows] = S z, with z's needed block columns already in LDS (zl).
// Each group keeps a running sum per row and stores it at seg[row + group];
// row `row` was touched exactly by groups rptr[row]/L .. (rptr[row+1]-1)/L,
// whose partials are then summed by 8 lanes per output (strided, then a
// 3-step butterfly): fixed order.
template <typename T, bool RES>
__device__ __forceinline__ void pcg_spmv_segments(const PcgArgs& a, int ib, int i0, int i1, const int* rptr,
                                                  PcgItems& it, const double* zl, double* seg) {
  const int g = threadIdx.x / 9, comp = threadIdx.x - 9 * (threadIdx.x / 9);
  if (g < SPMV_GROUPS) {
    double acc = 0.0;
    int cur = -1;
    for (int k0 = i0; k0 < i1; k0 += PCG_IPG) {
      if (!RES) pcg_load_items<T>(a, ib, k0, i1, rptr, comp, it);
#pragma unroll
      for (int kk = 0; kk < PCG_IPG; ++kk) {
        const int rl = it.rl[kk];
        if (rl < 0) continue;
        if (rl != cur) {
          if (cur >= 0) seg[(cur + g) * 9 + comp] = acc;
          acc = 0.0;
          cur = rl;
        }
        const double* zc = zl + it.lc[kk] * 9;
#pragma unroll
        for (int m = 0; m < 9; ++m) acc += it.v[kk][m] * zc[m];
      }
    }
    if (cur >= 0) seg[(cur + g) * 9 + comp] = acc;
  }
  __syncthreads();
}

// Output o of the product from the group partials (after
// pcg_spmv_segments): valid in every lane of each group of 8 lanes (sums
// over the group through DPP lane moves), for o = (base + threadIdx.x) / 8
// < nr * 9.
__device__ __forceinline__ double pcg_spmv_output(int o, int sub, int nr, int L, const int* rptr,
                                                  const double* seg) {
  double s = 0.0;
  if (o < nr * 9) {
    const int row = o / 9, cp = o - 9 * row;
    const int g0 = rptr[row] / L, g1 = (rptr[row + 1] - 1) / L;
    for (int gg = g0 + sub; gg <= g1; gg += 8) s += seg[(row + gg) * 9 + cp];
  }
  s += dpp_mov<0xB1, 0xF>(s);   // quad_perm [1,0,3,2]
  s += dpp_mov<0x4E, 0xF>(s);   // quad_perm [2,3,0,1]
  s += dpp_mov<0x141, 0xF>(s);  // row_half_mirror: the other quad of the 8
  return s;
}

template <typename T, bool RES>
__device__ __forceinline__ void pcg_spmv(const PcgArgs& a, int ib, int i0, int i1, int nr, int L,
                                         const int* rptr, PcgItems& it, const double* zl, double* seg,
                                         double* y) {
  pcg_spmv_segments<T, RES>(a, ib, i0, i1, rptr, it, zl, seg);
  const int nout = nr * 9;
  for (int base = 0; base < nout * 8; base += blockDim.x) {
    const int t = base + threadIdx.x, o = t >> 3, sub = t & 7;
    const double v = pcg_spmv_output(o, sub, nr, L, rptr, seg);
    if (o < nout && sub == 0) y[o] = v;
  }
  __syncthreads();
}

// fetch block columns cols[0 .. n) from ring slot zk into LDS (as D)
template <typename D>
__device__ __forceinline__ void fetch_cols(const int32_t* cols, const double* zk, int n, D* zl) {
  for (int u = threadIdx.x; u < n * 9; u += blockDim.x) {
    const int j = u / 9;
    zl[u] = (D)zk[(size_t)cols[j] * ZSTRIDE + (u - 9 * j)];
  }
}

// fetch the block columns this workgroup reads from ring slot zk into LDS
__device__ __forceinline__ void pcg_fetch_z(const PcgArgs& a, const double* zk, int ub, int nuc,
                                            double* zl) {
  fetch_cols(a.ucol + ub, zk, nuc, zl);
}

template <typename T, bool RES>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_standard(PcgArgs a) {
  __shared__ double xs[PCG_RMAX * 9], rs[PCG_RMAX * 9], ps[PCG_RMAX * 9];
  __shared__ double qs[PCG_RMAX * 9], zs[PCG_RMAX * 9], ys[PCG_RMAX * 9];
  __shared__ double Ml[PCG_RMAX * 81];
  __shared__ double zl[PCG_ZCOLS * 9];
  __shared__ double seg[(PCG_RMAX + SPMV_GROUPS) * 9];
  __shared__ int rptr[PCG_RMAX + 1];
  __shared__ double red[PCG_THREADS / 64];
  const int G = gridDim.x, B = xcd_block(blockIdx.x, gridDim.x), tid = threadIdx.x, nt = blockDim.x;
  const int r0 = a.wg_row[B], nr = a.wg_row[B + 1] - r0;
  const int n9 = nr * 9;
  const int ib = a.item_ptr[B], nitems = a.item_ptr[B + 1] - ib;
  const int ub = a.ucol_ptr[B], nuc = a.ucol_ptr[B + 1] - ub;
  const size_t zstride = (size_t)a.nc * ZSTRIDE, pstride = (size_t)G * PART_STRIDE;
  const int g = tid / 9, comp = tid - 9 * (tid / 9);
  const int L = max(1, (nitems + SPMV_GROUPS - 1) / SPMV_GROUPS);
  const int i0 = g < SPMV_GROUPS ? min(nitems, g * L) : nitems;
  const int i1 = g < SPMV_GROUPS ? min(nitems, i0 + L) : nitems;
  if (tid == 0) {
    rptr[0] = 0;
    for (int i = 0; i < nr; ++i)
      rptr[i + 1] = rptr[i] + (a.S_ptr[r0 + i + 1] - a.S_ptr[r0 + i]) +
                    (a.T_ptr[r0 + i + 1] - a.T_ptr[r0 + i]);
  }
  for (int i = tid; i < n9; i += nt) {
    rs[i] = a.b[9 * (size_t)r0 + i];
    xs[i] = 0.0;
  }
  for (int i = tid; i < nr * 81; i += nt) Ml[i] = a.Minv[81 * (size_t)r0 + i];
  __syncthreads();
  PcgItems it;
  if (RES && i0 < i1) pcg_load_items<T>(a, ib, i0, i1, rptr, comp, it);
  else {
#pragma unroll
    for (int kk = 0; kk < PCG_IPG; ++kk) it.rl[kk] = -1, it.lc[kk] = 0;
  }

  // z0 = M b, p0 = z0
  double s_bb = 0.0, s_rz = 0.0;
  for (int i = tid; i < n9; i += nt) {
    const int row = i / 9, cp = i - 9 * row;
    double z = 0.0;
#pragma unroll
    for (int m = 0; m < 9; ++m) z += Ml[row * 81 + cp * 9 + m] * rs[row * 9 + m];
    zs[i] = z;
    ps[i] = z;
    publish(a.zring + (size_t)(r0 + row) * ZSTRIDE + cp, z);
    s_bb += rs[i] * rs[i];
    s_rz += rs[i] * z;
  }
  s_bb = block_sum(s_bb, red);
  s_rz = block_sum(s_rz, red);
  if (tid == 0) {
    publish(a.partA + (size_t)B * PART_STRIDE, s_bb);
    publish(a.partA + (size_t)B * PART_STRIDE + 1, s_rz);
  }
  bool ok = grid_barrier(a.gs, a.error);
  pcg_fetch_z(a, a.zring, ub, nuc, zl);
  double t0 = 0.0, t1 = 0.0;
  for (int i = tid; i < G; i += nt) {
    t0 += a.partA[(size_t)i * PART_STRIDE];
    t1 += a.partA[(size_t)i * PART_STRIDE + 1];
  }
  const double bb = block_sum(t0, red);
  double rz = block_sum(t1, red);
  const double bnorm = sqrt(bb);
  double rnorm = bnorm;
  int iters = 0, breakdown = 0;
  if (ok && bnorm > 0.0) {
    // q0 = S z0 (= S p0)
    pcg_spmv<T, RES>(a, ib, i0, i1, nr, L, rptr, it, zl, seg, ys);
    double s_pq = 0.0;
    for (int i = tid; i < n9; i += nt) {
      qs[i] = ys[i];
      s_pq += ps[i] * ys[i];
    }
    s_pq = block_sum(s_pq, red);
    if (tid == 0) publish(a.partB + (size_t)B * PART_STRIDE, s_pq);
    ok = grid_barrier(a.gs, a.error);
    t0 = 0.0;
    for (int i = tid; i < G; i += nt) t0 += a.partB[(size_t)i * PART_STRIDE];
    double pq = block_sum(t0, red);
    if (ok && !(pq > 0.0)) breakdown = 1;
    double alpha = rz / pq;
    for (int k = 1; ok && !breakdown && k <= a.maxiter; ++k) {
      for (int i = tid; i < n9; i += nt) {
        xs[i] += alpha * ps[i];
        rs[i] -= alpha * qs[i];
      }
      __syncthreads();
      double* zk = a.zring + (size_t)k * zstride;
      double s_rr = 0.0, s_rz2 = 0.0;
      for (int i = tid; i < n9; i += nt) {
        const int row = i / 9, cp = i - 9 * row;
        double z = 0.0;
#pragma unroll
        for (int m = 0; m < 9; ++m) z += Ml[row * 81 + cp * 9 + m] * rs[row * 9 + m];
        zs[i] = z;
        publish(zk + (size_t)(r0 + row) * ZSTRIDE + cp, z);
        s_rr += rs[i] * rs[i];
        s_rz2 += rs[i] * z;
      }
      s_rr = block_sum(s_rr, red);
      s_rz2 = block_sum(s_rz2, red);
      double* pa = a.partA + (size_t)k * pstride;
      if (tid == 0) {
        publish(pa + (size_t)B * PART_STRIDE, s_rr);
        publish(pa + (size_t)B * PART_STRIDE + 1, s_rz2);
      }
      ok = grid_barrier(a.gs, a.error);
      if (!ok) break;
      // the partials and the z columns arrive in the same memory round trip
      pcg_fetch_z(a, zk, ub, nuc, zl);
      t0 = 0.0;
      t1 = 0.0;
      for (int i = tid; i < G; i += nt) {
        t0 += pa[(size_t)i * PART_STRIDE];
        t1 += pa[(size_t)i * PART_STRIDE + 1];
      }
      const double rr = block_sum(t0, red);
      const double rz_new = block_sum(t1, red);
      iters = k;
      rnorm = sqrt(rr);
      if (rnorm <= a.rtol * bnorm) break;
      const double beta = rz_new / rz;
      rz = rz_new;
      for (int i = tid; i < n9; i += nt) ps[i] = zs[i] + beta * ps[i];
      pcg_spmv<T, RES>(a, ib, i0, i1, nr, L, rptr, it, zl, seg, ys);
      s_pq = 0.0;
      for (int i = tid; i < n9; i += nt) {
        const double q = ys[i] + beta * qs[i];
        qs[i] = q;
        s_pq += ps[i] * q;
      }
      s_pq = block_sum(s_pq, red);
      double* pb = a.partB + (size_t)k * pstride;
      if (tid == 0) publish(pb + (size_t)B * PART_STRIDE, s_pq);
      ok = grid_barrier(a.gs, a.error);
      if (!ok) break;
      t0 = 0.0;
      for (int i = tid; i < G; i += nt) t0 += pb[(size_t)i * PART_STRIDE];
      pq = block_sum(t0, red);
      if (!(pq > 0.0)) {
        breakdown = 1;
        break;
      }
      alpha = rz / pq;
    }
  }
  for (int i = tid; i < n9; i += nt) a.x[9 * (size_t)r0 + i] = xs[i];
  if (B == 0 && tid == 0) {
    a.info->cg_iters = iters;
    a.info->cg_breakdown = breakdown;
    a.info->cg_rel_resid = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  }
}

// Pipelined PCG (Ghysels and Vanroose, "Hiding global synchronization
// latency in the preconditioned Conjugate Gradient algorithm", 2014): the
// same Krylov iterates as the standard recurrence in exact arithmetic, with
// the three dot products of an iteration reduced together and the product
// n = S m computed after the same barrier, so each iteration needs one grid
// barrier and one memory round trip.  Its attainable accuracy is lower than
// the standard recurrence's (relative residuals below ~1e-10 may not be
// reached), which is why the standard kernel stays selectable.
template <typename T, bool RES>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_pipelined(PcgArgs a) {
  __shared__ double xs[PCG_RMAX * 9], rs[PCG_RMAX * 9], us[PCG_RMAX * 9], ws[PCG_RMAX * 9];
  __shared__ double ms_[PCG_RMAX * 9], zs[PCG_RMAX * 9], qs[PCG_RMAX * 9];
  __shared__ double ss[PCG_RMAX * 9], ps[PCG_RMAX * 9];
  __shared__ double Ml[PCG_RMAX * 81];
  __shared__ double zl[PCG_ZCOLS * 9];
  __shared__ double seg[(PCG_RMAX + SPMV_GROUPS) * 9];
  __shared__ int rptr[PCG_RMAX + 1];
  __shared__ int ucl[PCG_ZCOLS];  // the block columns read (global index)
  __shared__ double red[PCG_THREADS / 64];
  const int G = gridDim.x, B = xcd_block(blockIdx.x, gridDim.x), tid = threadIdx.x, nt = blockDim.x;
  const int r0 = a.wg_row[B], nr = a.wg_row[B + 1] - r0;
  const int n9 = nr * 9;
  const int ib = a.item_ptr[B], nitems = a.item_ptr[B + 1] - ib;
  const int ub = a.ucol_ptr[B], nuc = a.ucol_ptr[B + 1] - ub;
  const size_t zstride = (size_t)a.nc * ZSTRIDE, pstride = (size_t)G * PART_STRIDE;
  const int g = tid / 9, comp = tid - 9 * (tid / 9);
  const int L = max(1, (nitems + SPMV_GROUPS - 1) / SPMV_GROUPS);
  const int i0 = g < SPMV_GROUPS ? min(nitems, g * L) : nitems;
  const int i1 = g < SPMV_GROUPS ? min(nitems, i0 + L) : nitems;
  if (tid == 0) {
    rptr[0] = 0;
    for (int i = 0; i < nr; ++i)
      rptr[i + 1] = rptr[i] + (a.S_ptr[r0 + i + 1] - a.S_ptr[r0 + i]) +
                    (a.T_ptr[r0 + i + 1] - a.T_ptr[r0 + i]);
  }
  // the recurrences of the first iteration read z, q, s, p with beta = 0:
  // they must hold zeros, not whatever the LDS held before (0 * NaN = NaN)
  for (int i = tid; i < n9; i += nt) {
    rs[i] = a.b[9 * (size_t)r0 + i];
    xs[i] = 0.0;
    zs[i] = 0.0;
    qs[i] = 0.0;
    ss[i] = 0.0;
    ps[i] = 0.0;
  }
  for (int i = tid; i < nr * 81; i += nt) Ml[i] = a.Minv[81 * (size_t)r0 + i];
  for (int j = tid; j < nuc; j += nt) ucl[j] = a.ucol[ub + j];
  __syncthreads();
  PcgItems it;
  if (RES && i0 < i1) pcg_load_items<T>(a, ib, i0, i1, rptr, comp, it);
  else {
#pragma unroll
    for (int kk = 0; kk < PCG_IPG; ++kk) it.rl[kk] = -1, it.lc[kk] = 0;
  }
  // u0 = M b, published in slot 0; w0 = S u0
  double s_bb = 0.0;
  for (int i = tid; i < n9; i += nt) {
    const int row = i / 9, cp = i - 9 * row;
    double u = 0.0;
#pragma unroll
    for (int m = 0; m < 9; ++m) u += Ml[row * 81 + cp * 9 + m] * rs[row * 9 + m];
    us[i] = u;
    publish(a.zring + (size_t)(r0 + row) * ZSTRIDE + cp, u);
    s_bb += rs[i] * rs[i];
  }
  s_bb = block_sum(s_bb, red);
  if (tid == 0) publish(a.partB + (size_t)B * PART_STRIDE, s_bb);
  // this workgroup's dot-product records of every iteration slot, and (with
  // register-resident blocks) its z columns of ring slots 1 .. maxiter + 1:
  // pending
  for (int q = tid; q < 3 * (a.maxiter + 1); q += nt)
    clear_record(a.partA + (size_t)(q / 3) * pstride + (size_t)B * PART_STRIDE + (q - 3 * (q / 3)));
  if (RES) {
    for (int q = tid; q < (a.maxiter + 1) * n9; q += nt) {
      const int sl = q / n9, k = q - sl * n9, row = k / 9;
      clear_record(a.zring + (size_t)(sl + 1) * zstride + (size_t)(r0 + row) * ZSTRIDE + (k - 9 * row));
    }
  }
  bool ok = grid_barrier(a.gs, a.error);
  fetch_cols(ucl, a.zring, nuc, zl);
  double t0 = 0.0;
  for (int i = tid; i < G; i += nt) t0 += a.partB[(size_t)i * PART_STRIDE];
  const double bnorm = sqrt(block_sum(t0, red));
  __shared__ int poll_failed;
  __shared__ double red3s[3 * (PCG_THREADS / 64)];
  if (tid == 0) poll_failed = 0;
  pcg_spmv<T, RES>(a, ib, i0, i1, nr, L, rptr, it, zl, seg, ws);
  double rnorm = bnorm, gamma_old = 1.0, alpha_old = 1.0;
  int iters = 0, breakdown = 0;
  if constexpr (RES) {
    // Thread tid < n9 owns element tid of the workgroup's rows (at most
    // PCG_RMAX * 9 < PCG_THREADS).  Wavefront 0 alone forms the step's
    // scalars, while the others start the product, and hands them over
    // through LDS with the product's barrier; the convergence test is read
    // there too (the last iteration's product is formed and dropped).
    const bool own = tid < n9;
    const int orow = own ? tid / 9 : 0, ocp = tid - 9 * (tid / 9);
    const unsigned zoff = (unsigned)(r0 + orow) * ZSTRIDE + (unsigned)ocp;
    const int nwa = (n9 + 63) >> 6;  // wavefronts holding elements
    const int nwr = (G + 63) >> 6;   // wavefronts polling dot records
    __shared__ double scal[5];       // alpha, beta, residual norm; previous gamma, alpha
    __shared__ int sstate;           // 0: continue, 1: converged or at maxiter, 2: breakdown
    for (int i = 0; ok && bnorm > 0.0 && i <= a.maxiter; ++i) {
      // local: partial dots of r, u, w; m = M w published in slot i + 1
      double* zk = a.zring + (size_t)(i + 1) * zstride;
      double s_g = 0.0, s_d = 0.0, s_r = 0.0;
      if (own) {
        double m = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) m += Ml[orow * 81 + ocp * 9 + q] * ws[orow * 9 + q];
        ms_[tid] = m;
        publish(zk + zoff, m);
        const double r = rs[tid], u = us[tid], w = ws[tid];
        s_g = r * u;
        s_d = w * u;
        s_r = r * r;
      }
      double* pa = a.partA + (size_t)i * pstride;
      if (nwa == 1) {
        // one wavefront holds every element: it publishes its sums itself
        if (tid < 64) {
          s_g = dpp_wave_total(s_g);
          s_d = dpp_wave_total(s_d);
          s_r = dpp_wave_total(s_r);
          if (tid == 63) {
            publish(pa + (size_t)B * PART_STRIDE, s_g);
            publish(pa + (size_t)B * PART_STRIDE + 1, s_d);
            publish(pa + (size_t)B * PART_STRIDE + 2, s_r);
          }
        }
      } else {
        __shared__ double red3[PCG_THREADS / 64][3];
        if ((tid >> 6) < nwa) {
          s_g = dpp_wave_total(s_g);
          s_d = dpp_wave_total(s_d);
          s_r = dpp_wave_total(s_r);
          if ((tid & 63) == 63) {
            red3[tid >> 6][0] = s_g;
            red3[tid >> 6][1] = s_d;
            red3[tid >> 6][2] = s_r;
          }
        }
        __syncthreads();
        if (tid < 3) {
          double v = 0.0;
          for (int w2 = 0; w2 < nwa; ++w2) v += red3[w2][tid];
          publish(pa + (size_t)B * PART_STRIDE + tid, v);
        }
      }
      // the z columns this workgroup reads and (thread t < G) workgroup t's
      // partials, in one poll; each polling wavefront sums its partials
      double tg = 0.0, td = 0.0, tr = 0.0;
      if (!poll_slot(ucl, nuc, zk, zl, tid < G ? pa + (size_t)tid * PART_STRIDE : nullptr, tg, td, tr,
                     a.error))
        poll_failed = 1;
      if ((tid >> 6) < nwr) {
        tg = dpp_wave_total(tg);
        td = dpp_wave_total(td);
        tr = dpp_wave_total(tr);
        if ((tid & 63) == 63) {
          red3s[3 * (tid >> 6)] = tg;
          red3s[3 * (tid >> 6) + 1] = td;
          red3s[3 * (tid >> 6) + 2] = tr;
        }
      }
      __syncthreads();
      if (poll_failed) {
        ok = false;
        break;
      }
      if (tid < 64) {
        // the wavefront sums in a fixed order: identical in every workgroup
        double gamma = 0.0, delta = 0.0, rr = 0.0;
        for (int w2 = 0; w2 < nwr; ++w2) {
          gamma += red3s[3 * w2];
          delta += red3s[3 * w2 + 1];
          rr += red3s[3 * w2 + 2];
        }
        gamma = uniform(gamma);
        delta = uniform(delta);
        rr = uniform(rr);
        const double rn = sqrt(rr);
        int st = 0;
        double alpha = 0.0, beta = 0.0;
        if (rn <= a.rtol * bnorm || i == a.maxiter) {
          st = 1;
        } else {
          beta = i > 0 ? gamma / scal[3] : 0.0;
          const double den = i > 0 ? delta - beta * gamma / scal[4] : delta;
          if (!(den > 0.0)) st = 2;
          else alpha = gamma / den;
        }
        if (tid == 0) {
          scal[0] = alpha;
          scal[1] = beta;
          scal[2] = rn;
          scal[3] = gamma;
          scal[4] = alpha;
          sstate = st;
        }
      }
      pcg_spmv_segments<T, RES>(a, ib, i0, i1, rptr, it, zl, seg);
      iters = i;
      if (sstate) {
        rnorm = scal[2];
        breakdown = sstate == 2;
        break;
      }
      const double alpha = scal[0], beta = scal[1];
      // n = S m, output by output, straight into the vector updates
      for (int base = 0; base < n9 * 8; base += nt) {
        const int t = base + tid, k = t >> 3, sub = t & 7;
        const double nk = pcg_spmv_output(k, sub, nr, L, rptr, seg);
        if (k < n9 && sub == 0) {
          const double z = nk + beta * zs[k];
          const double q = ms_[k] + beta * qs[k];
          const double sv = ws[k] + beta * ss[k];
          const double pv = us[k] + beta * ps[k];
          zs[k] = z;
          qs[k] = q;
          ss[k] = sv;
          ps[k] = pv;
          xs[k] += alpha * pv;
          rs[k] -= alpha * sv;
          us[k] -= alpha * q;
          ws[k] -= alpha * z;
        }
      }
      __syncthreads();
    }
  } else {
  for (int i = 0; ok && bnorm > 0.0 && i <= a.maxiter; ++i) {
    // local: partial dots of r, u, w; m = M w published in slot i + 1
    double* zk = a.zring + (size_t)(i + 1) * zstride;
    double s_g = 0.0, s_d = 0.0, s_r = 0.0;
    for (int k = tid; k < n9; k += nt) {
      const int row = k / 9, cp = k - 9 * row;
      double m = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) m += Ml[row * 81 + cp * 9 + q] * ws[row * 9 + q];
      ms_[k] = m;
      publish(zk + (size_t)(r0 + row) * ZSTRIDE + cp, m);
      s_g += rs[k] * us[k];
      s_d += ws[k] * us[k];
      s_r += rs[k] * rs[k];
    }
    s_g = wave_sum(s_g);
    s_d = wave_sum(s_d);
    s_r = wave_sum(s_r);
    __shared__ double red3[PCG_THREADS / 64][3];
    if ((tid & 63) == 0) {
      red3[tid >> 6][0] = s_g;
      red3[tid >> 6][1] = s_d;
      red3[tid >> 6][2] = s_r;
    }
    // the m columns must have reached memory before the partials are seen
    __builtin_amdgcn_s_waitcnt(0);
    if (tid == 0) poll_failed = 0;
    __syncthreads();
    double* pa = a.partA + (size_t)i * pstride;
    if (tid < 3) {
      double v = 0.0;
      for (int w2 = 0; w2 < PCG_THREADS / 64; ++w2) v += red3[w2][tid];
      publish(pa + (size_t)B * PART_STRIDE + tid, v);
    }
    double tg = 0.0, td = 0.0, tr = 0.0;
    if (tid < G && !poll_record(pa + (size_t)tid * PART_STRIDE, tg, td, tr, a.error)) poll_failed = 1;
    // the workgroup partials summed in a fixed order (wavefront butterflies,
    // then the wavefronts in order), one exchange that is also the barrier
    // after the poll
    tg = wave_sum(tg);
    td = wave_sum(td);
    tr = wave_sum(tr);
    if ((tid & 63) == 0) {
      red3s[3 * (tid >> 6)] = tg;
      red3s[3 * (tid >> 6) + 1] = td;
      red3s[3 * (tid >> 6) + 2] = tr;
    }
    __syncthreads();
    if (poll_failed) {
      ok = false;
      break;
    }
    // every workgroup's m columns are in memory now
    fetch_cols(ucl, zk, nuc, zl);
    double gamma = 0.0, delta = 0.0, rr = 0.0;
#pragma unroll 2
    for (int w2 = 0; w2 < PCG_THREADS / 64; ++w2) {
      gamma += red3s[3 * w2];
      delta += red3s[3 * w2 + 1];
      rr += red3s[3 * w2 + 2];
    }
    // (identical in every thread: scalar registers)
    gamma = uniform(gamma);
    delta = uniform(delta);
    rr = uniform(rr);
    iters = i;
    rnorm = sqrt(rr);
    if (rnorm <= a.rtol * bnorm || i == a.maxiter) break;
    const double beta = i > 0 ? gamma / gamma_old : 0.0;
    const double den = i > 0 ? delta - beta * gamma / alpha_old : delta;
    if (!(den > 0.0)) {
      breakdown = 1;
      break;
    }
    const double alpha = gamma / den;
    __syncthreads();  // zl complete
    pcg_spmv_segments<T, RES>(a, ib, i0, i1, rptr, it, zl, seg);
    // n = S m, output by output, straight into the vector updates
    for (int base = 0; base < n9 * 8; base += nt) {
      const int t = base + tid, k = t >> 3, sub = t & 7;
      const double nk = pcg_spmv_output(k, sub, nr, L, rptr, seg);
      if (k < n9 && sub == 0) {
        const double z = nk + beta * zs[k];
        const double q = ms_[k] + beta * qs[k];
        const double sv = ws[k] + beta * ss[k];
        const double pv = us[k] + beta * ps[k];
        zs[k] = z;
        qs[k] = q;
        ss[k] = sv;
        ps[k] = pv;
        xs[k] += alpha * pv;
        rs[k] -= alpha * sv;
        us[k] -= alpha * q;
        ws[k] -= alpha * z;
      }
    }
    __syncthreads();
    gamma_old = gamma;
    alpha_old = alpha;
  }
  }
  for (int i = tid; i < n9; i += nt) a.x[9 * (size_t)r0 + i] = xs[i];
  if (B == 0 && tid == 0) {
    a.info->cg_iters = iters;
    a.info->cg_breakdown = breakdown;
    a.info->cg_rel_resid = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  }
}

// ---------------------------------------------------------------------------
// Pipelined PCG with streamed blocks (plans whose block rows do not fit the
// lanes' registers, e.g. the 10,000-camera scene).  Each upper off-diagonal
// block S_ab (a < b) is read once per product, by the workgroup that owns row
// a, from a copy in the storage precision T padded to SI_STRIDE values
// (written by the Schur kernel; a workgroup's blocks contiguous in row
// order).  These plans have their own row decomposition, balanced by upper
// blocks.
//
// The blocks are split into StreamShape<T>::groups contiguous ranges,
// StreamShape<T>::wave_groups nine-lane groups per wavefront (6 for FP32
// blocks, 3 for FP64: either way a wavefront stages 126 16-byte pieces per
// step).  At each step a wavefront stages the current block of each of its
// groups in LDS with 16-byte loads (the next two steps' blocks in flight),
// and lane `comp` of a group forms from the one staged block
//   (S_ab v_b)[comp]    (row comp): running sum of row a, per (row + group)
//                       segment as in the resident kernels;
//   (S_ab^T v_a)[comp]  (column comp): added to the workgroup's LDS sum for
//                       block column b (one per distinct column).
// The column sums of the workgroup's own rows join its row sums; the others
// go to the owner of b through a write-once exchange slot per (workgroup,
// column) and product, after which the workgroup raises its flag of that
// product.  An owner waits for the flags of the workgroups that send to it
// and adds their slots in a fixed order.  The LDS column sums take their
// terms in arrival order, so the last bits of a product may differ from run
// to run.
//
// The FP64 diagonal blocks are applied by the thread that owns each vector
// element.  Thread k owns element k of the workgroup's rows and keeps r, u,
// w, m, z, q and its row of the block-Jacobi factor in registers, x, p and s
// in LDS; w, m and the product n also pass through LDS.
// ---------------------------------------------------------------------------
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct StreamShape {
  static constexpr int wave_groups = sizeof(T) == 4 ? 6 : 3;  // nine-lane groups per wavefront
  static constexpr int groups = (PCG_THREADS / 64) * wave_groups;
  static constexpr int pieces = SI_STRIDE * (int)sizeof(T) / 16;  // 16-byte pieces per block
  static constexpr int loads = (wave_groups * pieces + 63) / 64;
};
constexpr int STREAM_LOADS = 2;
static_assert(StreamShape<float>::loads == STREAM_LOADS && StreamShape<double>::loads == STREAM_LOADS,
              "both block precisions stage two 16-byte pieces per lane and step");
constexpr int STREAM_GROUPS_MAX = StreamShape<float>::groups;
// a wavefront's staging area holds every piece its lanes move, so that the
// LDS stores need no lane-dependent branch (such a branch inside the
// lockstep loop lets the compiler restructure it into a divergent nest)
// With FP32 blocks the staged blocks of groups 4 and 5 start one 16-byte
// piece later than packed: the lanes of a wavefront half then read the rows
// and columns of their groups' blocks with fewer LDS bank conflicts (3 passes
// per read instead of 4, for 32 banks of 4 bytes).  One spare piece per
// wavefront holds the shift of the lane pieces past the blocks.
constexpr int STREAM_SKEW_GROUP = 4;
constexpr int STREAM_WAVE_BYTES = (STREAM_LOADS * 64 + 1) * 16;
template <typename T>
__device__ __forceinline__ int stream_piece(int p) {
  return sizeof(T) == 4 && p >= STREAM_SKEW_GROUP * (SI_STRIDE * 4 / 16) ? p + 1 : p;
}
template <typename T>
__device__ __forceinline__ int stream_group_offset(int gl) {
  return gl * SI_STRIDE + (sizeof(T) == 4 && gl >= STREAM_SKEW_GROUP ? 4 : 0);
}

// wait until the exchange flag at f (one sender, one product) is raised
__device__ __forceinline__ bool poll_flag(const double* f, int* error) {
  const unsigned long long* r = reinterpret_cast<const unsigned long long*>(f);
  long spins = 0;
  while (__hip_atomic_load(r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == PCG_PENDING) {
    if (++spins > BARRIER_SPIN_LIMIT ||
        (__hip_atomic_load(error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_BARRIER)) {
      atomicOr(error, (int)ERR_BARRIER);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// threadIdx.x passed through an empty asm statement: address arithmetic
// derived from it is redone where it is used instead of being hoisted out of
// the CG loop.  Hoisted, those per-lane addresses outlive the registers and
// are spilled to scratch, and the wait for each reload also waits for every
// load issued before it (the next product's block prefetch among them).
__device__ __forceinline__ int fresh_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Per-workgroup constants of the streamed product.
struct StreamCtx {
  int B, G, r0, nr, sib, nitems, L, vb, nvc, ib, src;  // src: this thread's sender (t < senders)
  size_t vbase;
};

// Lane `lane` of wavefront `wave` loads piece (64 j + lane) % pieces
// of the step-k block of group (64 j + lane) / pieces of its
// wavefront; loads are issued without branches (items clamped to the
// workgroup's last one).  The workgroup must have items.
template <typename T>
__device__ __forceinline__ void stream_fetch(const PcgArgs& a, const StreamCtx& c,
                                             f32x4_t (&buf)[STREAM_LOADS], int k) {
  using Sh = StreamShape<T>;
  const int tx = fresh_tid(), wave = tx >> 6, lane = tx & 63;
  const unsigned char* __restrict__ SIb =
      reinterpret_cast<const unsigned char*>(a.SI) + (size_t)c.sib * SI_STRIDE * sizeof(T);
#pragma unroll
  for (int j = 0; j < STREAM_LOADS; ++j) {
    const int q = 64 * j + lane;
    const int gg = min(q / Sh::pieces, Sh::wave_groups - 1), pc = q % Sh::pieces;
    const int item = min(min(c.nitems, (wave * Sh::wave_groups + gg) * c.L) + k, c.nitems - 1);
    buf[j] = *reinterpret_cast<const f32x4_t*>(SIb + (size_t)item * (SI_STRIDE * sizeof(T)) + pc * 16);
  }
}

// nl[k] = (S v)[row k / 9 of the workgroup, component k % 9] without the
// diagonal block, k < nr * 9, for the block columns of v in zl (the columns
// vcl of the workgroup's upper blocks) and its own rows in ml; product
// `slot` of the solve (exchange slot and flag).  The received column sums of
// row i are listed at ipl[i] .. ipl[i+1] (the first STREAM_IN_MAX in inl).
// The blocks of steps 0 and 1 are in A and Bf on entry (loaded by the caller
// or by the previous product, the blocks being the same); on exit they hold
// them again for the next product.  After the blocks, the owning thread's
// row of the block-Jacobi factor is loaded into Mr (its latency hidden by
// the exchange).  Every thread of the workgroup calls it (barriers inside);
// tl must be zero on entry and is zero on exit.
template <typename T>
__device__ __forceinline__ bool stream_spmv(const PcgArgs& a, const StreamCtx& c, int slot,
                                            const int* rptr, const int* lcol, const int* vcl,
                                            const int* ipl, const int* inl, const double* zl,
                                            const double* ml, double* tl, double* seg,
                                            unsigned char* st, double* nl, int* poll_failed,
                                            double (&Mr)[9], f32x4_t (&A)[STREAM_LOADS],
                                            f32x4_t (&Bf)[STREAM_LOADS], const double* rec,
                                            unsigned long long (&rv)[3]) {
  using Sh = StreamShape<T>;
  const int tx = fresh_tid(), wave = tx >> 6, lane = tx & 63;
  const int gl = lane / 9, comp = lane - 9 * gl;
  const bool computes = gl < Sh::wave_groups;
  const int g = wave * Sh::wave_groups + gl;
  const int nitems = c.nitems, L = c.L;
  const int i0 = computes ? min(nitems, g * L) : nitems;
  const int i1 = computes ? min(nitems, i0 + L) : nitems;
  unsigned char* wst = st + wave * STREAM_WAVE_BYTES;
  if (nitems > 0) {
    const int* __restrict__ scol = a.sitem_col + c.sib;
    auto fetch = [&](f32x4_t (&buf)[STREAM_LOADS], int k) { stream_fetch<T>(a, c, buf, k); };
    auto stage = [&](const f32x4_t (&buf)[STREAM_LOADS]) {
#pragma unroll
      for (int j = 0; j < STREAM_LOADS; ++j)
        *reinterpret_cast<f32x4_t*>(wst + stream_piece<T>(64 * j + lane) * 16) = buf[j];
    };
    double acc = 0.0;
    int cur = -1, row = 0;
    auto multiply = [&](int k, int col) {
      __builtin_amdgcn_wave_barrier();
      const int ik = i0 + k;
      if (computes && ik < i1) {
        while (rptr[row + 1] <= ik) ++row;
        if (row != cur) {
          if (cur >= 0) seg[(cur + g) * 9 + comp] = acc;
          acc = 0.0;
          cur = row;
        }
        const T* blk = reinterpret_cast<const T*>(wst + stream_group_offset<T>(gl) * sizeof(T));
        const double* zc = zl + col * 9;
        const double* va = ml + row * 9;
#pragma unroll
        for (int m = 0; m < 9; ++m) acc += (double)blk[comp * 9 + m] * zc[m];
        // (the two products one after the other: fewer live registers)
        __builtin_amdgcn_sched_barrier(0);
        double t = 0.0;
#pragma unroll
        for (int m = 0; m < 9; ++m) t += (double)blk[m * 9 + comp] * va[m];
        atomicAdd(tl + col * 9 + comp, t);
      }
      __builtin_amdgcn_wave_barrier();
    };
    // the blocks of steps k + 1 and k + 2 in flight while step k is
    // multiplied (past the last step the last one is loaded again, never
    // staged)
    int col = scol[min(i0, nitems - 1)];
    stage(A);
    for (int k = 0; k < L; k += 2) {
      // (when L is odd the last pass's second half multiplies nothing:
      // every group's range ends by step L - 1)
      fetch(A, min(k + 2, L - 1));
      int col_next = scol[min(i0 + k + 1, nitems - 1)];
      multiply(k, col);
      if (k + 1 < L) stage(Bf);
      col = col_next;
      fetch(Bf, min(k + 3, L - 1));
      col_next = scol[min(i0 + k + 2, nitems - 1)];
      multiply(k + 1, col);
      if (k + 2 < L) stage(A);
      col = col_next;
    }
    // the first two steps of the next product
    fetch(A, 0);
    fetch(Bf, min(1, L - 1));
    if (cur >= 0) seg[(cur + g) * 9 + comp] = acc;
  }
  __syncthreads();
  const int nout = c.nr * 9;
  {
    // (assigned in every thread: the previous values are dead here)
    const int o = min(tx, nout - 1);
    const size_t q = 81 * (size_t)(c.r0 + o / 9) + 9 * (o % 9);
#pragma unroll
    for (int k = 0; k < 9; ++k) Mr[k] = a.Minv[q + k];
  }
  // column sums of other workgroups' rows to their exchange slots
  double* rk = a.rring + (size_t)slot * a.rstride + c.vbase;
  for (int u = tx; u < c.nvc * 9; u += blockDim.x) {
    const int j = u / 9, b = vcl[j];
    if (b < c.r0 || b >= c.r0 + c.nr) publish(rk + u, tl[u]);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tx == 0) publish(a.rflag + (size_t)slot * c.G + c.B, 1.0);
  // outputs: the groups rptr[row] / L .. (rptr[row + 1] - 1) / L touched row
  // `row` (none when the row has no upper block); 8 lanes per output,
  // strided then three DPP lane moves: fixed order; then the row's own
  // column sum, when one of the workgroup's blocks lies in its column
  for (int base = 0; base < nout * 8; base += blockDim.x) {
    const int t = base + tx, o = t >> 3, sub = t & 7;
    double sum = 0.0;
    int row = 0, cp = 0;
    if (o < nout) {
      row = o / 9;
      cp = o - 9 * row;
      if (rptr[row + 1] > rptr[row]) {
        const int g0 = rptr[row] / L, g1 = (rptr[row + 1] - 1) / L;
        for (int gg = g0 + sub; gg <= g1; gg += 8) sum += seg[(row + gg) * 9 + cp];
      }
    }
    sum += dpp_mov<0xB1, 0xF>(sum);   // quad_perm [1,0,3,2]
    sum += dpp_mov<0x4E, 0xF>(sum);   // quad_perm [2,3,0,1]
    sum += dpp_mov<0x141, 0xF>(sum);  // row_half_mirror: the other quad of the 8
    if (o < nout && sub == 0) nl[o] = lcol[row] >= 0 ? sum + tl[lcol[row] * 9 + cp] : sum;
  }
  // the three words at rec (a dot record, when given), read once while the
  // senders' flags are awaited: write-once words, so a value that is not
  // pending is final (the caller polls again for a pending one)
  if (rec) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
      rv[q] = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(rec) + q, __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
  }
  // wait for the workgroups that send to this one (thread t for sender t)
  if (c.src >= 0 && !poll_flag(a.rflag + (size_t)slot * c.G + c.src, a.error)) *poll_failed = 1;
  __syncthreads();
  // their slots, in the fixed order of each row's list; tl cleared
  if (!*poll_failed && tx < nout) {
    const int row = tx / 9, cp = tx - 9 * row;
    const double* rs = a.rring + (size_t)slot * a.rstride + cp;
    const int k0 = ipl[row], k1 = ipl[row + 1];
    double sum = 0.0;
#pragma unroll 4
    for (int k = k0; k < k1; ++k) sum += rs[k < STREAM_IN_MAX ? inl[k] : a.in_off[c.ib + k]];
    nl[tx] += sum;
  }
  for (int u = tx; u < c.nvc * 9; u += blockDim.x) tl[u] = 0.0;
  __syncthreads();
  return *poll_failed == 0;
}

template <typename T>
__global__ __launch_bounds__(PCG_THREADS) void k_pcg_stream(PcgArgs a) {
  __shared__ double zl[STREAM_COLS * 9], tl[STREAM_COLS * 9];
  // w and the product n of the owned elements live in zl's memory: w is read
  // (m = M w) before the columns are fetched, n is written after the blocks
  // have been multiplied and read before the next fetch
  double* const wl = zl;
  double* const nl = zl + STREAM_RMAX * 9;
  __shared__ double ml[STREAM_RMAX * 9];
  // x, p and s of the owned elements (owner thread only: fewer live
  // registers across the product)
  __shared__ double xl[STREAM_RMAX * 9], pl[STREAM_RMAX * 9], sl[STREAM_RMAX * 9];
  __shared__ double seg[(STREAM_RMAX + STREAM_GROUPS_MAX) * 9];
  __shared__ __align__(16) unsigned char st[(PCG_THREADS / 64) * STREAM_WAVE_BYTES];
  __shared__ int rptr[STREAM_RMAX + 1], lcol[STREAM_RMAX], ipl[STREAM_RMAX + 1];
  __shared__ int vcl[STREAM_COLS], inl[STREAM_IN_MAX];
  __shared__ double red[PCG_THREADS / 64];
  __shared__ double red3[PCG_THREADS / 64][3];
  __shared__ double red3s[3 * (PCG_THREADS / 64)];
  __shared__ double scal[5];  // alpha, beta, residual norm; previous gamma, alpha (wavefront 0)
  __shared__ int sstate;      // 0: continue, 1: converged or at maxiter, 2: breakdown
  __shared__ int poll_failed;
  const int G = gridDim.x, B = xcd_block(blockIdx.x, gridDim.x), tid = threadIdx.x, nt = blockDim.x;
  StreamCtx c;
  c.B = B;
  c.G = G;
  c.r0 = a.wg_row[B];
  c.nr = a.wg_row[B + 1] - c.r0;
  c.sib = a.sitem_ptr[B];
  c.nitems = a.sitem_ptr[B + 1] - c.sib;
  c.L = max(1, (c.nitems + StreamShape<T>::groups - 1) / StreamShape<T>::groups);
  c.vb = a.vcol_ptr[B];
  c.nvc = a.vcol_ptr[B + 1] - c.vb;
  c.vbase = (size_t)a.vbase[B];
  c.ib = a.in_ptr[c.r0];
  {
    const int s0 = a.src_ptr[B], ns = a.src_ptr[B + 1] - s0;
    c.src = tid < ns ? a.src[s0 + tid] : -1;
  }
  const int r0 = c.r0, nr = c.nr, n9 = nr * 9;
  const size_t zstride = (size_t)a.nc * ZSTRIDE, pstride = (size_t)G * PART_STRIDE;
  // the first two steps' blocks of every product, loaded early
  f32x4_t A[STREAM_LOADS], Bf[STREAM_LOADS];
  if (c.nitems > 0) {
    stream_fetch<T>(a, c, A, 0);
    stream_fetch<T>(a, c, Bf, min(1, c.L - 1));
  }
  if (tid == 0) {
    rptr[0] = 0;
    for (int i = 0; i < nr; ++i) rptr[i + 1] = rptr[i] + (a.S_ptr[r0 + i + 1] - a.S_ptr[r0 + i] - 1);
    poll_failed = 0;
  }
  for (int i = tid; i < nr; i += nt) lcol[i] = -1;
  for (int i = tid; i <= nr; i += nt) ipl[i] = a.in_ptr[r0 + i] - c.ib;
  for (int k = tid; k < min(a.in_ptr[r0 + nr] - c.ib, STREAM_IN_MAX); k += nt) inl[k] = a.in_off[c.ib + k];
  for (int j = tid; j < c.nvc; j += nt) vcl[j] = a.vcol[c.vb + j];
  for (int u = tid; u < c.nvc * 9; u += nt) tl[u] = 0.0;
  __syncthreads();
  for (int j = tid; j < c.nvc; j += nt) {
    const int b = vcl[j];
    if (b >= r0 && b < r0 + nr) lcol[b - r0] = j;
  }
  // thread tid owns element tid of the workgroup's rows; Mr holds its row
  // of the block-Jacobi factor, drow points to its row of the FP64 diagonal
  // block (read when applied, while the workgroups synchronise)
  const bool own = tid < n9;
  const int row = own ? tid / 9 : 0, cp = own ? tid - 9 * row : 0;
  double r = 0.0, u = 0.0, w = 0.0, m = 0.0, z = 0.0, q = 0.0;
  const double* drow = a.Sdiag + 81 * (size_t)(r0 + row) + cp * 9;
  double Mr[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Mr[k] = own ? a.Minv[81 * (size_t)(r0 + row) + cp * 9 + k] : 0.0;
  if (own) {
    r = a.b[9 * (size_t)r0 + tid];
    nl[tid] = r;
    xl[tid] = 0.0;
    pl[tid] = 0.0;
    sl[tid] = 0.0;
  }
  __syncthreads();
  // u0 = M b, published in slot 0; w0 = S u0
  double s_bb = 0.0;
  if (own) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) v += Mr[k] * nl[row * 9 + k];
    u = v;
    ml[tid] = u;
    publish(a.zring + (size_t)(r0 + row) * ZSTRIDE + cp, u);
    s_bb = r * r;
  }
  s_bb = block_sum(s_bb, red);  // (its barriers also complete ml)
  if (tid == 0) publish(a.partB + (size_t)B * PART_STRIDE, s_bb);
  double nd = 0.0;  // diagonal part of the product
  if (own) {
#pragma unroll
    for (int k = 0; k < 9; ++k) nd += drow[k] * ml[row * 9 + k];
  }
  for (int k = tid; k < 3 * (a.maxiter + 1); k += nt)
    clear_record(a.partA + (size_t)(k / 3) * pstride + (size_t)B * PART_STRIDE + (k - 3 * (k / 3)));
  for (int k = tid; k < a.maxiter + 2; k += nt) clear_record(a.rflag + (size_t)k * G + B);
  // The z columns of this workgroup's rows are marked pending before their
  // ring slot is read (readers poll them together with the dot records):
  // slots 1 .. 3 here; slot i + 3 by each element's owner in iteration i,
  // which the product's wait for its stores before it raises its flag
  // completes before any workgroup can reach iteration i + 2, where slot
  // i + 3 is read; the owner's own value store to it comes later in program
  // order.
  for (int k = tid; k < min(3, a.maxiter + 1) * n9; k += nt) {
    const int sl = k / n9, e = k - sl * n9, rw = e / 9;
    clear_record(a.zring + (size_t)(sl + 1) * zstride + (size_t)(r0 + rw) * ZSTRIDE + (e - 9 * rw));
  }
  bool ok = grid_barrier(a.gs, a.error);
  fetch_cols(vcl, a.zring, c.nvc, zl);
  double t0 = 0.0;
  for (int i = tid; i < G; i += nt) t0 += a.partB[(size_t)i * PART_STRIDE];
  const double bnorm = uniform(sqrt(block_sum(t0, red)));  // (its barriers complete zl)
  unsigned long long rv[3];
  if (ok) ok = stream_spmv<T>(a, c, 0, rptr, lcol, vcl, ipl, inl, zl, ml, tl, seg, st, nl, &poll_failed, Mr, A, Bf,
                              nullptr, rv);
  if (own) {
    w = nl[tid] + nd;
    wl[tid] = w;
  }
  __syncthreads();
  double rnorm = bnorm;
  int iters = 0, breakdown = 0;
  const int nwr = (G + 63) >> 6;  // wavefronts polling dot records
  for (int i = 0; ok && bnorm > 0.0 && i <= a.maxiter; ++i) {
    // local: partial dots of r, u, w; m = M w published in slot i + 1
    double* zk = a.zring + (size_t)(i + 1) * zstride;
    double s_g = 0.0, s_d = 0.0, s_r = 0.0;
    if (own) {
      if (i + 3 <= a.maxiter + 1) clear_record(zk + 2 * zstride + (size_t)(r0 + row) * ZSTRIDE + cp);
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 9; ++k) v += Mr[k] * wl[row * 9 + k];
      m = v;
      ml[tid] = m;
      publish(zk + (size_t)(r0 + row) * ZSTRIDE + cp, m);
      s_g = r * u;
      s_d = w * u;
      s_r = r * r;
    }
    const int nwa = (n9 + 63) >> 6;  // wavefronts holding elements
    if ((tid >> 6) < nwa) {
      s_g = dpp_wave_total(s_g);
      s_d = dpp_wave_total(s_d);
      s_r = dpp_wave_total(s_r);
      if ((tid & 63) == 63) {
        red3[tid >> 6][0] = s_g;
        red3[tid >> 6][1] = s_d;
        red3[tid >> 6][2] = s_r;
      }
    }
    __syncthreads();
    double* pa = a.partA + (size_t)i * pstride;
    if (tid < 3) {
      double v = 0.0;
      for (int w2 = 0; w2 < nwa; ++w2) v += red3[w2][tid];
      publish(pa + (size_t)B * PART_STRIDE + tid, v);
    }
    // the diagonal part of n = S m while the other workgroups catch up
    nd = 0.0;
    if (own) {
#pragma unroll
      for (int k = 0; k < 9; ++k) nd += drow[k] * ml[row * 9 + k];
    }
    // the m columns this workgroup reads (into zl: w is no longer needed in
    // its memory) and (thread t < G) workgroup t's dot partials.  The product
    // n = S m needs no scalar of this iteration: with FP32 blocks it is formed
    // before the partials of all workgroups are read (the grid-wide
    // reduction waits behind the streaming, the partials are read during the
    // product's exchange, and the last iteration's product is formed and
    // dropped); with FP64 blocks the columns and partials are polled
    // together and the product follows the scalars (each order measured the
    // faster one for its precision)
    constexpr bool defer = sizeof(T) == 4;
    double tg = 0.0, td = 0.0, tr = 0.0;
    const double* rec = tid < G ? pa + (size_t)tid * PART_STRIDE : nullptr;
    if (!poll_slot(vcl, c.nvc, zk, zl, defer ? nullptr : rec, tg, td, tr, a.error)) poll_failed = 1;
    if constexpr (defer) {
      __syncthreads();
      if (poll_failed) {
        ok = false;
        break;
      }
      if (!stream_spmv<T>(a, c, i + 1, rptr, lcol, vcl, ipl, inl, zl, ml, tl, seg, st, nl, &poll_failed, Mr, A, Bf,
                          rec, rv)) {
        ok = false;
        break;
      }
      // partials still pending when read are polled
      if (rec) {
        if (rv[0] != PCG_PENDING && rv[1] != PCG_PENDING && rv[2] != PCG_PENDING) {
          tg = __longlong_as_double((long long)rv[0]);
          td = __longlong_as_double((long long)rv[1]);
          tr = __longlong_as_double((long long)rv[2]);
        } else if (!poll_slot(vcl, 0, zk, zl, rec, tg, td, tr, a.error)) {
          poll_failed = 1;
        }
      }
    }
    // each polling wavefront sums its partials
    if ((tid >> 6) < nwr) {
      tg = dpp_wave_total(tg);
      td = dpp_wave_total(td);
      tr = dpp_wave_total(tr);
      if ((tid & 63) == 63) {
        red3s[3 * (tid >> 6)] = tg;
        red3s[3 * (tid >> 6) + 1] = td;
        red3s[3 * (tid >> 6) + 2] = tr;
      }
    }
    __syncthreads();
    if (poll_failed) {
      ok = false;
      break;
    }
    if (tid < 64) {
      // the step's scalars, in wavefront 0 only (the wavefront sums in a
      // fixed order: identical in every workgroup)
      double gamma = 0.0, delta = 0.0, rr = 0.0;
      for (int w2 = 0; w2 < nwr; ++w2) {
        gamma += red3s[3 * w2];
        delta += red3s[3 * w2 + 1];
        rr += red3s[3 * w2 + 2];
      }
      gamma = uniform(gamma);
      delta = uniform(delta);
      rr = uniform(rr);
      const double rn = sqrt(rr);
      int st_ = 0;
      double al = 0.0, be = 0.0;
      if (rn <= a.rtol * bnorm || i == a.maxiter) {
        st_ = 1;
      } else {
        be = i > 0 ? gamma / scal[3] : 0.0;
        const double den = i > 0 ? delta - be * gamma / scal[4] : delta;
        if (!(den > 0.0)) st_ = 2;
        else al = gamma / den;
      }
      if (tid == 0) {
        scal[0] = al;
        scal[1] = be;
        scal[2] = rn;
        scal[3] = gamma;
        scal[4] = al;
        sstate = st_;
      }
    }
    __syncthreads();  // the scalars
    iters = i;
    if (sstate) {
      rnorm = scal[2];
      breakdown = sstate == 2;
      break;
    }
    const double alpha = scal[0], beta = scal[1];
    if constexpr (!defer) {
      if (!stream_spmv<T>(a, c, i + 1, rptr, lcol, vcl, ipl, inl, zl, ml, tl, seg, st, nl, &poll_failed, Mr, A,
                          Bf, nullptr, rv)) {
        ok = false;
        break;
      }
    }
    if (own) {
      const int t2 = fresh_tid();
      const double n = nl[t2] + nd;
      z = n + beta * z;
      q = m + beta * q;
      const double s = w + beta * sl[t2];
      sl[t2] = s;
      const double p = u + beta * pl[t2];
      pl[t2] = p;
      xl[t2] += alpha * p;
      r -= alpha * s;
      u -= alpha * q;
      w -= alpha * z;
      wl[t2] = w;
    }
    __syncthreads();
  }
  if (own) a.x[9 * (size_t)r0 + tid] = xl[tid];
  if (B == 0 && tid == 0) {
    a.info->cg_iters = iters;
    a.info->cg_breakdown = breakdown;
    a.info->cg_rel_resid = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
static const void* pcg_kernel(bool resident, bool pipelined, bool stream) {
  if (pipelined && !resident && stream) return reinterpret_cast<const void*>(k_pcg_stream<T>);
  if (pipelined)
    return resident ? reinterpret_cast<const void*>(k_pcg_pipelined<T, true>)
                    : reinterpret_cast<const void*>(k_pcg_pipelined<T, false>);
  return resident ? reinterpret_cast<const void*>(k_pcg_standard<T, true>)
                  : reinterpret_cast<const void*>(k_pcg_standard<T, false>);
}

template <typename T>
int pcg_max_grid(bool resident, bool pipelined, bool stream) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, pcg_kernel<T>(resident, pipelined, stream),
                                                   PCG_THREADS, 0) != hipSuccess)
    return 0;
  return ncu * per;
}
template int pcg_max_grid<float>(bool, bool, bool);
template int pcg_max_grid<double>(bool, bool, bool);

// The streamed kernel runs when the arguments carry the streamed
// decomposition (pipelined recurrence, blocks not register-resident); such
// plans without it read the stored blocks per item.
template <typename T>
hipError_t launch_pcg(const PcgArgs& a, int grid, bool resident, bool pipelined, hipStream_t s) {
  const bool stream = pipelined && !resident && a.SI;
  if (stream && (!a.sitem_ptr || !a.sitem_col || !a.vcol_ptr || !a.vcol || !a.vbase || !a.in_ptr ||
                 !a.in_off || !a.src_ptr || !a.src || !a.rring || !a.rflag))
    return hipErrorInvalidValue;  // the streamed kernel needs its decomposition and exchange
  void* args[] = {const_cast<PcgArgs*>(&a)};
  return hipLaunchCooperativeKernel(pcg_kernel<T>(resident, pipelined, stream), dim3(grid),
                                    dim3(PCG_THREADS), args, 0, s);
}
template hipError_t launch_pcg<float>(const PcgArgs&, int, bool, bool, hipStream_t);
template hipError_t launch_pcg<double>(const PcgArgs&, int, bool, bool, hipStream_t);

}  // namespace ba
