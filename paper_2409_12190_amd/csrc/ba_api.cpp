// C ABI of the bundle-adjustment library: problem lifetime, workspace
// carving, the LM iteration driver and read-back.  See include/ba.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "ba.h"
#include "ba_adjoint.h"
#include "ba_dense.h"
#include "ba_internal.h"
#include "ba_kernels.h"
#include "ba_pgo.h"
#include "ba_precond.h"

// A training graph: the camera pattern (host) and its device view.
struct ba_graph {
  int nc = 0;
  int64_t nnzb = 0;
  std::vector<int32_t> nbr_ptr, nbr, rev;
  size_t ws_needed = 0;
  bool bound = false;
  hipStream_t stream = nullptr;
  ba::GraphDev dev{};
};

namespace {

thread_local std::string g_err;

ba_status fail(ba_status s, const std::string& m) {
  g_err = m;
  return s;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(BA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

struct Carver {
  char* base;
  size_t off = 0;
  size_t last = 0;  // offset of the most recent region
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    last = off;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += std::max<size_t>(n, 1) * sizeof(T);
    return p;
  }
};

size_t elem_bytes(const ba_problem* p) { return p->opt.precision == BA_MIXED ? 4 : 8; }

// the chunks of points seen more than CHUNK times (their own kernels)
ba::LongChunks long_chunks(const ba_problem* p) {
  return ba::LongChunks{p->b.long_chunk, (int)p->plan.long_chunk.size()};
}

void carve(ba_problem* p, char* base, size_t* total) {
  Carver c{base};
  const ba::Plan& P = p->plan;
  ba::Buffers& b = p->b;
  const size_t nc = P.nc, nnzb = P.nnzb;
  // a pose graph keeps its plan's observation and point tables (two
  // observations per edge) but none of their values
  const size_t np = p->pgo ? 0 : P.np, no = p->pgo ? 0 : P.no;
  const size_t nch = std::max<size_t>(P.chunk_ptr.size() - 1, (size_t)ba::pgo_chunks(p->n_edges));
  const size_t es = elem_bytes(p);
  b.o_cam = c.take<int32_t>(P.o_cam.size());
  b.o_pt = c.take<int32_t>(P.o_pt.size());
  b.pt_ptr = c.take<int32_t>(P.pt_ptr.size());
  b.chunk_ptr = c.take<int32_t>(nch + 1);
  b.chunk_pt = c.take<int32_t>(nch + 1);
  b.long_chunk = c.take<int32_t>(P.long_chunk.size());
  b.cam_ptr = c.take<int32_t>(nc + 1);
  b.cam_obs = c.take<int32_t>(P.cam_obs.size());
  b.S_ptr = c.take<int32_t>(nc + 1);
  b.S_col = c.take<int32_t>(nnzb);
  b.T_ptr = c.take<int32_t>(nc + 1);
  b.T_blk = c.take<int32_t>(P.T_blk.size());
  b.T_src = c.take<int32_t>(P.T_src.size());
  b.pair_x = c.take<int32_t>(P.n_pairs);
  b.pair_y = c.take<int32_t>(P.n_pairs);
  b.slot_blk = c.take<int32_t>(P.slot_blk.size());
  b.slot_pb = c.take<int32_t>(P.slot_pb.size());
  b.slot_pe = c.take<int32_t>(P.slot_pe.size());
  b.slot_lead = c.take<int32_t>(P.slot_lead.size());
  b.stab = c.take<int32_t>(P.stab.size());
  b.swptr = c.take<int32_t>(P.swptr.size());
  b.blk_row = c.take<int32_t>(nnzb);
  b.pcg_row = c.take<int32_t>(P.pcg_row.size());
  b.item_ptr = c.take<int32_t>(P.item_ptr.size());
  b.item_e = c.take<int32_t>(P.item_e.size());
  b.item_code = c.take<int32_t>(P.item_code.size());
  b.ucol_ptr = c.take<int32_t>(P.ucol_ptr.size());
  b.ucol = c.take<int32_t>(P.ucol.size());
  b.srow = c.take<int32_t>(P.srow.size());
  b.sitem_ptr = c.take<int32_t>(P.sitem_ptr.size());
  b.sitem_col = c.take<int32_t>(P.sitem_col.size());
  b.blk_pos = c.take<int32_t>(P.blk_pos.size());
  b.vcol_ptr = c.take<int32_t>(P.vcol_ptr.size());
  b.vcol = c.take<int32_t>(P.vcol.size());
  b.vbase = c.take<int32_t>(P.vbase.size());
  b.in_ptr = c.take<int32_t>(P.in_ptr.size());
  b.in_off = c.take<int32_t>(P.in_off.size());
  b.src_ptr = c.take<int32_t>(P.src_ptr.size());
  b.src = c.take<int32_t>(P.src.size());
  b.o_orig = c.take<int64_t>(P.o_orig.size());
  b.fixed = c.take<uint8_t>(nc);
  b.o_xy = c.take<double>(2 * no);
  b.o_w = c.take<double>(no);
  for (int i = 0; i < 2; ++i) {
    b.cams[i] = c.take<double>(10 * nc);
    b.pts[i] = c.take<double>(3 * np);
  }
  b.r = c.take<double>(2 * no);
  b.w = c.take<double>(no);
  // observation rows, then the records (in the same 64-byte units: the Schur
  // step table addresses both from J; 32 doubles of padding after the last
  // record, which the staging reads past)
  b.J = c.take<char>(no * ba::NJ * es);
  const size_t off_J = c.last;
  b.rec = c.take<double>(8 * no + 32);
  p->rec_off = c.last - off_J;
  b.V = c.take<double>(6 * np);
  b.gp = c.take<double>(3 * np);
  b.gc = c.take<double>(9 * nc);
  b.diagU = c.take<double>(9 * nc);
  b.Vinv = c.take<double>(6 * np);
  b.ep = c.take<double>(3 * np);
  b.S = c.take<char>(nnzb * 81 * es);
  // streamed PCG plans (pipelined recurrence): one copy of each upper
  // off-diagonal block in the storage precision, the column-sum exchange
  const bool stream = !P.pcg_resident && P.sgrid > 0 && p->opt.cg_variant == BA_CG_PIPELINED &&
                      p->opt.linear_solver == BA_SOLVER_PCG;
  b.SI = c.take<char>(stream ? P.sitem_col.size() * ba::SI_STRIDE * es : 0);
  b.Sdiag = c.take<double>(81 * nc);
  b.bS = c.take<double>(9 * nc);
  b.Minv = c.take<double>(81 * nc);
  b.x = c.take<double>(9 * nc);
  b.dp = c.take<double>(3 * np);
  b.part_cost = c.take<double>(nch);
  b.part_cost_new = c.take<double>(nch);
  b.part_pred = c.take<double>(2 * nch);
  b.part_gmax = c.take<double>(nch);
  b.part_linc = c.take<double>((nc + 255) / 256);
  b.part_stage = c.take<double>(4 * ba::FINAL_STAGE_MAX);
  const size_t slots = (size_t)p->opt.cg_maxiter + 2;
  b.zring = c.take<double>(slots * nc * ba::ZSTRIDE);
  b.partA = c.take<double>(slots * std::max(P.pcg_grid, P.sgrid) * ba::PART_STRIDE);
  b.partB = c.take<double>(slots * std::max(P.pcg_grid, P.sgrid) * ba::PART_STRIDE);
  b.rring = c.take<double>(stream ? slots * (size_t)P.rstride : 0);
  b.rflag = c.take<double>(stream ? slots * (size_t)P.sgrid : 0);
  if (p->opt.linear_solver == BA_SOLVER_CHOLESKY) {
    const size_t ld = ba::dense_ld(P.nc), n = 9 * nc;
    b.dA = c.take<double>((n + 1) * ld);
    b.dLinv = c.take<double>(ld / ba::DENSE_NB * ba::DENSE_NB * ba::DENSE_NB);
    b.dpart = c.take<double>((n + ba::DENSE_BROWS - 1) / ba::DENSE_BROWS * ba::DENSE_NB);
    b.dresid = c.take<double>(2 * nc);
  }
  b.dev = c.take<ba::DevScalars>(1);
  b.dinfo = c.take<ba_step_info>(1);
  b.gsync = c.take<ba::GridSync>(1);
  if (p->opt.enable_backward) {
    b.adjA = c.take<double>(78 * no);
    b.adjJ = c.take<double>(24 * no);
    b.adjY = c.take<double>(27 * no);
    b.adjU = c.take<double>(81 * nc);
    b.adjS = es == 8 ? reinterpret_cast<double*>(b.S) : c.take<double>(81 * nnzb);
    b.adj_gt = c.take<double>(9 * nc);
    b.adj_vc = c.take<double>(9 * nc);
    b.adj_vp = c.take<double>(3 * np);
    b.adj_dev = c.take<ba::DevScalars>(1);
    b.adj_stat = c.take<double>(2);
    b.adj_info = c.take<ba_step_info>(1);
  }
  if (p->opt.precond == BA_PRECOND_LEARNED) {
    const size_t ns = P.nbr.size();
    b.pcLinv = c.take<double>(81 * nc);
    b.pcMinvL = c.take<double>(81 * nc);
    b.pc_params = c.take<float>(ba::GNN_NPARAM);
    b.pc_wbf16 = c.take<short>(ba::GNN_NBF16);
    b.nbr_ptr = c.take<int32_t>(nc + 1);
    b.nbr = c.take<int32_t>(ns);
    b.nbr_blk = c.take<int32_t>(ns);
    b.nbr_rev = c.take<int32_t>(ns);
    b.gX = c.take<float>(nc * ba::GNN_F);
    b.gE = c.take<float>(nc * 45);
    b.gw = c.take<float>(ns);
    b.gact = c.take<float>((2 * (ba::GNN_L + 1) + ba::GNN_L) * nc * ba::GNN_H);
  }
  b.cam_perm = c.take<int32_t>(p->reordered ? nc : 0);
  b.adj_gcam = c.take<double>(p->reordered && p->opt.enable_backward ? 10 * nc : 0);
  if (p->pgo) {
    const size_t m = p->n_edges;
    b.pg_ei = c.take<int32_t>(m);
    b.pg_ej = c.take<int32_t>(m);
    b.pg_ptr = c.take<int32_t>(p->pg_ptr.size());
    b.pg_code = c.take<int32_t>(p->pg_code.size());
    b.pg_T = c.take<double>(8 * m);
    b.pg_om = c.take<double>(36 * m);
    b.pg_rec = c.take<double>(ba::PGO_REC * m);
  }
  *total = c.off + 256;
}

template <class T>
hipError_t upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// Problems bound to the static scratch of a device: the one that holds it
// now (a later ba_problem_bind_static on the same device takes it over).
std::mutex g_static_mu;
const ba_problem* g_static_owner[64] = {};

bool static_owner_is(const ba_problem* p) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  return p->device >= 0 && p->device < 64 && g_static_owner[p->device] == p;
}

// bound, and (for the static scratch) still its holder
bool usable(const ba_problem* p) { return p->bound && (!p->static_ws || static_owner_is(p)); }

const char* not_bound_msg(const ba_problem* p) {
  return p->bound ? "the device's static scratch was taken over by another problem"
                  : "problem is not bound to a workspace";
}

ba_status require_ready(const ba_problem* p) {
  if (!p) return fail(BA_EINVAL, "null problem");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  if (!p->have_obs) return fail(BA_ESTATE, p->pgo ? "measurements are not set" : "observations are not set");
  if (!p->have_params) return fail(BA_ESTATE, p->pgo ? "poses are not set" : "parameters are not set");
  return BA_OK;
}

// Device rows of per-camera values between caller order and the internal
// order: to_caller gathers internal rows into caller order, otherwise the
// caller's rows are scattered into internal order; `width` values of rows
// of src_stride / dst_stride doubles.
hipError_t copy_cameras(const ba_problem* p, const double* src, int src_stride, double* dst, int dst_stride,
                        int width, bool to_caller) {
  const int nc = p->plan.nc;
  if (!p->reordered)
    return hipMemcpy2DAsync(dst, dst_stride * sizeof(double), src, src_stride * sizeof(double),
                            width * sizeof(double), nc, hipMemcpyDeviceToDevice, p->stream);
  ba::PermArgs a{nc, p->b.cam_perm, to_caller, src, dst, src_stride, dst_stride, width};
  return ba::launch_permute_rows(a, p->stream);
}

// Host rows (per camera, `width` values) from internal to caller order.
void rows_to_caller(const ba_problem* p, const double* in, double* out, size_t width) {
  const size_t nc = p->plan.nc;
  for (size_t c = 0; c < nc; ++c) {
    const size_t ic = p->reordered ? (size_t)p->cam_perm[c] : c;
    std::memcpy(out + c * width, in + ic * width, width * sizeof(double));
  }
}

// points held in the parameter state (none for a pose graph)
size_t point_count(const ba_problem* p) { return p->pgo ? 0 : (size_t)p->plan.np; }

// Event-bracketed launch of one phase when profiling is on.
struct Phase {
  ba_problem* p;
  int id;
  Phase(ba_problem* pp, int i) : p(pp), id(i) {
    if (on()) (void)hipEventRecord(p->ev[id][0], p->stream);
  }
  ~Phase() {
    if (on()) {
      (void)hipEventRecord(p->ev[id][1], p->stream);
      p->phase_used[id] = true;
    }
  }
  bool on() const { return p->profiling && (p->profile_mask >> id & 1u); }
};

void collect_phase_times(ba_problem* p) {
  if (!p->profiling) return;
  for (int i = 0; i < BA_NUM_PHASES; ++i) {
    if (!p->phase_used[i]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev[i][0], p->ev[i][1]) == hipSuccess) {
      p->phase_ms[i] += ms;
      p->phase_n[i] += 1;
    }
    p->phase_used[i] = false;
  }
}

#define PHASE(id, call)          \
  do {                           \
    Phase ph_(p, id);            \
    HIPCHK(call);                \
  } while (0)

// Graph view of the learned preconditioner's buffers inside a problem
// (inference only: no gradient buffers).
ba::GraphDev problem_graph(const ba_problem* p) {
  const ba::Buffers& b = p->b;
  ba::GraphDev g{};
  g.nc = p->plan.nc;
  g.ns = (int)p->plan.nbr.size();
  g.nbr_ptr = b.nbr_ptr;
  g.nbr = b.nbr;
  g.rev = b.nbr_rev;
  g.X = b.gX;
  g.E = b.gE;
  g.w = b.gw;
  const size_t blk = (size_t)g.nc * ba::GNN_H;
  float* a = b.gact;
  for (int l = 0; l <= ba::GNN_L; ++l) {
    g.Z[l] = a;
    a += blk;
    g.H[l] = a;
    a += blk;
  }
  for (int l = 0; l < ba::GNN_L; ++l) {
    g.M[l] = a;
    a += blk;
  }
  return g;
}

// Clears the PCG grid-barrier counters (a second PCG launch in one step).
hipError_t reset_sync(ba_problem* p) {
  return hipMemsetAsync(p->b.gsync, 0, sizeof(ba::GridSync), p->stream);
}

// plans whose pipelined PCG streams its blocks (a copy of each upper
// off-diagonal block, in the storage precision, written by the Schur kernel)
bool streamed(const ba_problem* p) {
  return !p->plan.pcg_resident && p->plan.sgrid > 0 && p->opt.cg_variant == BA_CG_PIPELINED &&
         p->opt.linear_solver == BA_SOLVER_PCG;
}

template <typename T>
ba_status lm_step_impl(ba_problem* p, ba_step_info* out) {
  using namespace ba;
  const Plan& P = p->plan;
  Buffers& b = p->b;
  hipStream_t s = p->stream;
  const int nchunk = p->pgo ? pgo_chunks(p->n_edges) : (int)P.chunk_ptr.size() - 1;
  const int cur = p->cur, nxt = p->cur ^ 1;
  const double lam_before = p->lambda;

  if (p->pgo) {
    // pose graph: per-edge residuals, Jacobians and records, then the
    // damped system's blocks straight from the records (no points)
    if (!p->lin_valid) {
      PgoLinArgs la{p->n_edges, b.pg_ei, b.pg_ej, b.cams[cur], b.pg_T, b.pg_om, b.pg_rec, b.part_cost,
                    b.part_gmax};
      PHASE(0, launch_pgo_linearize(la, s));
      PHASE(1, launch_reduce_cost(b.part_cost, nchunk, b.dev, s));
    }
    PgoAsmArgs aa{b.blk_row, b.S_col, b.pg_ptr, b.pg_code, b.fixed, b.pg_rec, b.S, b.Sdiag, b.gc, b.bS,
                  b.diagU, streamed(p) ? b.blk_pos : nullptr, streamed(p) ? b.SI : nullptr};
    PHASE(5, launch_pgo_assemble<T>(aa, P.nnzb, s));
  } else if (!p->lin_valid) {
    // linearisation with the point elimination of the current lambda
    LinArgs la{b.chunk_ptr, b.chunk_pt, b.pt_ptr, b.o_cam, b.o_pt, b.fixed, b.o_xy, b.o_w,
               b.cams[cur], b.pts[cur], p->opt.huber_delta, b.w, b.J, b.V, b.gp,
               b.part_cost, b.part_gmax, b.rec, p->opt.diag_min, p->opt.diag_max, b.Vinv, b.ep,
               b.dev, b.gsync};
    PHASE(0, launch_linearize<T>(la, nchunk, long_chunks(p), s));
    PHASE(1, launch_reduce_cost(b.part_cost, nchunk, b.dev, s));
  } else {
    // same linearisation, new lambda (after a rejected step): damp again
    DampArgs da{P.np, b.V, b.gp, p->opt.diag_min, p->opt.diag_max, b.Vinv, b.ep, b.dev, b.gsync};
    PHASE(2, launch_damp_points(da, s));
    PointQArgs qa{P.no, b.o_pt, b.w, b.Vinv, b.ep, b.J, b.rec};
    PHASE(3, launch_point_q<T>(qa, s));
  }
  if (!p->pgo) {
    // the camera vectors (gradient, right-hand side term, diag U) come from
    // the self pairs of the Schur kernel's diagonal blocks
    SchurArgs sa{P.n_schur_wg, p->rec_unit, b.slot_blk, b.slot_lead, b.blk_row, b.S_ptr, b.stab, b.swptr,
                 b.J, b.S, b.Sdiag, b.gc, b.bS, b.diagU};
    if (streamed(p)) {
      sa.blk_pos = b.blk_pos;
      sa.SI = b.SI;
    }
    PHASE(5, launch_schur_pairs<T>(sa, P.n_schur_wg, s));
  }
  CamFinishArgs cf{b.Sdiag, b.diagU, p->opt.diag_min, p->opt.diag_max, b.Minv, b.dev, b.pcLinv, b.gc, b.bS};
  PHASE(6, launch_camera_finish<T>(cf, P.nc, s));
  p->have_system = true;
  const bool learned = p->opt.precond == BA_PRECOND_LEARNED && p->gnn_ready;
  int32_t precond_used = 0;
  if (learned) {
    const GraphDev gd = problem_graph(p);
    PcFeatureArgs fa{P.nc, b.nbr_ptr, b.nbr, b.nbr_blk, b.S, b.pcLinv, b.gX, b.gE, b.gw, b.pc_params,
                     gd.H[0]};
    auto infer = [&]() -> hipError_t {
      hipError_t e = launch_pc_features<T>(fa, s);
      if (e == hipSuccess) e = launch_gnn_forward_bf16(gd, b.pc_params, b.pc_wbf16, s);
      if (e == hipSuccess) e = launch_gnn_output(gd, b.pc_params, b.pcLinv, b.pcMinvL, false, s);
      return e;
    };
    PHASE(12, infer());
    precond_used = 1;
  }
  PcgArgs pa{P.nc, p->cg_maxiter, p->cg_rtol, b.S_ptr, b.T_ptr, b.pcg_row, b.item_ptr, b.item_e,
             b.item_code, b.ucol_ptr, b.ucol, b.S, b.Sdiag, learned ? b.pcMinvL : b.Minv, b.bS, b.x,
             b.zring, b.partA, b.partB, b.dinfo, b.gsync, &b.dev->error};
  const bool pipe = p->opt.cg_variant == BA_CG_PIPELINED;
  int pcg_grid = P.pcg_grid;
  if (streamed(p)) {
    pa.wg_row = b.srow;
    pa.sitem_ptr = b.sitem_ptr;
    pa.sitem_col = b.sitem_col;
    pa.SI = b.SI;
    pa.vcol_ptr = b.vcol_ptr;
    pa.vcol = b.vcol;
    pa.vbase = b.vbase;
    pa.in_ptr = b.in_ptr;
    pa.in_off = b.in_off;
    pa.src_ptr = b.src_ptr;
    pa.src = b.src;
    pa.rstride = P.rstride;
    pa.rring = b.rring;
    pa.rflag = b.rflag;
    pcg_grid = P.sgrid;
  }
  if (p->opt.linear_solver == BA_SOLVER_CHOLESKY) {
    DenseArgs da{P.nc, P.nnzb, (int64_t)dense_ld(P.nc), b.dA, b.dLinv, b.dpart, b.dresid, b.x, b.bS,
                 b.Sdiag, b.S, b.S_ptr, b.S_col, b.blk_row, b.T_ptr, b.T_blk, b.T_src, b.dinfo,
                 &b.dev->error};
    PHASE(7, launch_dense_solve<T>(da, s));
  } else {
    PHASE(7, launch_pcg<T>(pa, pcg_grid, P.pcg_resident, pipe, s));
  }
  if (learned) {
    // the learned blocks are trusted unless their PCG failed: a breakdown,
    // a non-finite residual, or no reduction of the unpreconditioned
    // residual at all; then the step is solved again with block-Jacobi.  A
    // learned solve that reaches the iteration cap is an inexact step like
    // any other (the trust region judges it).
    HIPCHK(hipMemcpyAsync(p->hinfo, b.dinfo, sizeof(ba_step_info), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const ba_step_info& li = *p->hinfo;
    if (li.cg_breakdown || !(li.cg_rel_resid < 1.0)) {
      pa.Minv = b.Minv;
      HIPCHK(reset_sync(p));
      PHASE(7, launch_pcg<T>(pa, pcg_grid, P.pcg_resident, pipe, s));
      precond_used = 2;
    }
  }
  if (p->pgo) {
    RetractArgs ra{P.nc, b.fixed, b.cams[cur], b.x, b.gc, b.cams[nxt], b.part_linc};
    PHASE(9, launch_retract_cameras(ra, p->cam_blocks, s));
    PgoCandArgs ca{p->n_edges, b.pg_ei, b.pg_ej, b.cams[nxt], b.pg_T, b.pg_om, b.pg_rec, b.x,
                   b.part_cost_new, b.part_pred};
    PHASE(10, launch_pgo_candidate(ca, s));
  } else {
    BackArgs ba_{b.chunk_ptr, b.chunk_pt, b.pt_ptr, b.o_cam, b.o_pt, b.J, b.w, b.x, b.gp, b.Vinv,
                 b.pts[cur], b.dp, b.pts[nxt], b.part_pred};
    PHASE(8, launch_backsub<T>(ba_, nchunk, long_chunks(p), s));
    RetractArgs ra{P.nc, b.fixed, b.cams[cur], b.x, b.gc, b.cams[nxt], b.part_linc};
    PHASE(9, launch_retract_cameras(ra, p->cam_blocks, s));
    CostArgs co{b.chunk_ptr, b.o_cam, b.o_pt, b.o_xy, b.o_w, b.cams[nxt], b.pts[nxt],
                p->opt.huber_delta, b.part_cost_new};
    PHASE(10, launch_candidate_cost(co, nchunk, s));
  }
  FinalArgs fa{nchunk, p->cam_blocks, P.nc, b.part_cost_new, b.part_pred, b.part_linc, b.part_gmax,
               b.gc, p->opt.lambda_min, p->opt.lambda_max, b.dev, b.dinfo, b.part_stage, 0};
  PHASE(11, launch_finalize(fa, s));
  HIPCHK(hipMemcpyAsync(p->hinfo, b.dinfo, sizeof(ba_step_info), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(p->hscal, b.dev, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  collect_phase_times(p);

  ba_step_info info = *p->hinfo;
  info.precond_used = precond_used;
  info.stop_reason = BA_STOP_NONE;
  const int32_t err = p->hscal->error;
  if (err != 0 || !std::isfinite(info.cost_before)) {
    // leave theta and lambda as they were
    DevScalars restore{info.cost_before, lam_before, 0, 0};
    *p->hscal = restore;
    HIPCHK(hipMemcpyAsync(b.dev, p->hscal, sizeof(DevScalars), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    info.accepted = 0;
    info.lambda_next = lam_before;
    info.status = BA_ENUMERIC;
    if (out) *out = info;
    if (err & ERR_BARRIER) {
      info.status = BA_EHIP;
      if (out) *out = info;
      return fail(BA_EHIP, "the PCG grid barrier timed out");
    }
    std::string why = !std::isfinite(info.cost_before) ? "non-finite cost at the current parameters"
                      : (err & ERR_POINT_BLOCK)        ? "a damped point block is not positive definite"
                      : p->pgo                         ? "a damped diagonal pose block is not positive definite"
                                                       : "a diagonal camera block is not positive definite";
    return fail(BA_ENUMERIC, why);
  }
  p->lin_valid = true;
  if (info.accepted) {
    p->cur = nxt;
    p->lin_valid = false;
  }
  p->lambda = info.lambda_next;
  if (out) *out = info;
  return BA_OK;
}

void graph_carve(ba_graph* g, char* base, size_t* total) {
  Carver c{base};
  const size_t nc = g->nc, ns = g->nbr.size(), blk = nc * ba::GNN_H;
  ba::GraphDev& d = g->dev;
  d.nc = g->nc;
  d.ns = (int)ns;
  d.nbr_ptr = c.take<int32_t>(nc + 1);
  d.nbr = c.take<int32_t>(ns);
  d.rev = c.take<int32_t>(ns);
  d.X = c.take<float>(nc * ba::GNN_F);
  d.E = c.take<float>(nc * 45);
  d.w = c.take<float>(ns);
  for (int l = 0; l <= ba::GNN_L; ++l) {
    d.Z[l] = c.take<float>(blk);
    d.H[l] = c.take<float>(blk);
  }
  for (int l = 0; l < ba::GNN_L; ++l) d.M[l] = c.take<float>(blk);
  d.dO = c.take<float>(nc * ba::GNN_O);
  d.dH = c.take<float>(blk);
  d.dZ = c.take<float>(blk);
  d.dM = c.take<float>(blk);
  d.loss_part = c.take<double>(nc);
  d.loss = c.take<double>(1);
  *total = c.off + 256;
}

}  // namespace

namespace {

// Option checks shared by bundle-adjustment and pose-graph problems.
ba_status check_options(const ba_options& o, int32_t n_cams) {
  if (o.precision != BA_FP64 && o.precision != BA_MIXED) return fail(BA_EINVAL, "unknown precision");
  if (!(o.cg_rtol >= 0.0) || o.cg_maxiter < 1) return fail(BA_EINVAL, "bad CG options");
  if (o.cg_variant != BA_CG_PIPELINED && o.cg_variant != BA_CG_STANDARD)
    return fail(BA_EINVAL, "unknown CG variant");
  if (!(o.lambda0 > 0.0) || !(o.lambda_min > 0.0) || !(o.lambda_max >= o.lambda_min))
    return fail(BA_EINVAL, "bad damping options");
  if (!(o.diag_min > 0.0) || !(o.diag_max >= o.diag_min)) return fail(BA_EINVAL, "bad clamp range");
  if (o.precond != BA_PRECOND_BLOCK_JACOBI && o.precond != BA_PRECOND_LEARNED)
    return fail(BA_EINVAL, "unknown preconditioner");
  if (!(o.adjoint_grad_tol >= 0.0)) return fail(BA_EINVAL, "adjoint_grad_tol must be >= 0");
  if (o.linear_solver != BA_SOLVER_PCG && o.linear_solver != BA_SOLVER_CHOLESKY)
    return fail(BA_EINVAL, "unknown linear solver");
  if (o.linear_solver == BA_SOLVER_CHOLESKY && (n_cams > ba::DENSE_MAX_CAMS || o.precond == BA_PRECOND_LEARNED))
    return fail(BA_EUNSUPPORTED, "the dense Cholesky solve takes at most 2048 cameras and no learned preconditioner");
  if (o.camera_order != BA_ORDER_BANDWIDTH && o.camera_order != BA_ORDER_GIVEN)
    return fail(BA_EINVAL, "unknown camera order");
  return BA_OK;
}

// The internal camera numbering of a problem (identity unless the options
// ask for the bandwidth order and it differs from the caller's); returns
// the indices relabelled.
std::vector<int32_t> set_order(ba_problem* p, int32_t nc, int32_t np, int64_t no, const int32_t* cidx,
                               const int32_t* pidx) {
  std::vector<int32_t> perm;
  if (p->opt.camera_order == BA_ORDER_BANDWIDTH && nc > 1) perm = ba::camera_order(nc, np, no, cidx, pidx);
  bool ident = true;
  for (int32_t c = 0; c < (int32_t)perm.size() && ident; ++c) ident = perm[c] == c;
  std::vector<int32_t> out(cidx, cidx + no);
  if (perm.empty() || ident) return out;
  p->reordered = true;
  p->cam_perm = perm;
  p->cam_inv.assign(nc, 0);
  for (int32_t c = 0; c < nc; ++c) p->cam_inv[perm[c]] = c;
  for (int64_t k = 0; k < no; ++k) out[k] = perm[cidx[k]];
  return out;
}

// The block pattern in caller order (for ba_export of a renumbered problem).
void caller_pattern(ba_problem* p) {
  const ba::Plan& P = p->plan;
  const int32_t nc = P.nc;
  std::vector<std::vector<std::pair<int32_t, int32_t>>> rows(nc);  // (column, internal block)
  for (int32_t a = 0; a < nc; ++a)
    for (int32_t e = P.S_ptr[a]; e < P.S_ptr[a + 1]; ++e) {
      const int32_t ca = p->cam_inv[a], cb = p->cam_inv[P.S_col[e]];
      if (ca <= cb) rows[ca].push_back({cb, e});
      else rows[cb].push_back({ca, -1 - e});
    }
  p->x_ptr.assign(nc + 1, 0);
  p->x_col.clear();
  p->x_blk.clear();
  p->x_tr.clear();
  for (int32_t a = 0; a < nc; ++a) {
    auto& r = rows[a];
    std::sort(r.begin(), r.end());  // the diagonal (column a) comes first: no column below a
    for (const auto& cb : r) {
      p->x_col.push_back(cb.first);
      p->x_blk.push_back(cb.second >= 0 ? cb.second : -1 - cb.second);
      p->x_tr.push_back(cb.second < 0 ? 1 : 0);
    }
    p->x_ptr[a + 1] = (int64_t)p->x_col.size();
  }
}

// Sizes the workspace and the Schur step table of a planned problem; takes
// ownership of p (deleted on failure).
ba_status finish_create(ba_problem* p, ba_problem** out) {
  const ba_options& o = p->opt;
  if (p->reordered) {
    try {
      caller_pattern(p);
    } catch (const std::bad_alloc&) {
      delete p;
      return fail(BA_EINVAL, "out of host memory");
    }
  }
  p->lambda = o.lambda0;
  p->cg_rtol = o.cg_rtol;
  p->cg_maxiter = o.cg_maxiter;
  p->cam_blocks = (p->plan.nc + 255) / 256;
  carve(p, nullptr, &p->ws_needed);
  // Schur step table in 64-byte units from J: observation x's row at x * row
  // units, its record (self pairs, y side) at rec_unit + x, -1 unchanged
  const int64_t row_units = (int64_t)ba::NJ * (int64_t)elem_bytes(p) / 64;
  const int64_t rec_unit = (int64_t)(p->rec_off / 64);
  if (rec_unit + (int64_t)p->plan.no > INT32_MAX || p->rec_off % 64) {
    delete p;
    return fail(BA_EUNSUPPORTED, "observation rows exceed 2^31 units");
  }
  p->rec_unit = (int32_t)rec_unit;
  try {
    p->stab_units.resize(p->plan.stab.size());
  } catch (const std::bad_alloc&) {
    delete p;
    return fail(BA_EINVAL, "out of host memory");
  }
  for (size_t i = 0; i < p->stab_units.size(); ++i) {
    const int32_t c = p->plan.stab[i];
    p->stab_units[i] = c >= 0 ? (int32_t)(c * row_units) : (c == -1 ? -1 : (int32_t)(rec_unit + (-2 - c)));
  }
  *out = p;
  return BA_OK;
}

}  // namespace

extern "C" {

void ba_default_options(ba_options* o) {
  if (!o) return;
  o->cam_dof = 9;
  o->precision = BA_FP64;
  o->huber_delta = 0.0;
  o->cg_rtol = 1e-4;
  o->cg_maxiter = 250;
  o->lambda0 = 1e-4;
  o->lambda_min = 1e-12;
  o->lambda_max = 1e12;
  o->diag_min = 1e-6;
  o->diag_max = 1e32;
  o->cg_variant = BA_CG_PIPELINED;
  o->enable_backward = 0;
  o->adjoint_rtol = 1e-10;
  o->precond = BA_PRECOND_BLOCK_JACOBI;
  o->adjoint_grad_tol = 1e-6;
  o->linear_solver = BA_SOLVER_PCG;
  o->camera_order = BA_ORDER_BANDWIDTH;
}

const char* ba_last_error(void) { return g_err.c_str(); }

ba_status ba_problem_create(const ba_options* opt, int32_t n_cams, int32_t n_pts, int64_t n_obs,
                            const int32_t* cam_idx, const int32_t* pt_idx, ba_problem** out) {
  if (!out) return fail(BA_EINVAL, "out is null");
  *out = nullptr;
  if (!cam_idx || !pt_idx) return fail(BA_EINVAL, "index arrays must not be null");
  ba_options o;
  if (opt) o = *opt;
  else ba_default_options(&o);
  if (o.cam_dof != 9 && o.cam_dof != 6) return fail(BA_EUNSUPPORTED, "cam_dof must be 9 or 6");
  if (o.cam_dof == 6 && (o.precond == BA_PRECOND_LEARNED || o.enable_backward))
    return fail(BA_EUNSUPPORTED, "the 6-DoF camera supports neither the learned preconditioner nor the adjoint");
  const ba_status st = check_options(o, n_cams);
  if (st != BA_OK) return st;
  if (n_cams <= 0 || n_pts <= 0 || n_obs <= 0) return fail(BA_EINVAL, "n_cams, n_pts and n_obs must be positive");
  for (int64_t k = 0; k < n_obs; ++k)
    if (cam_idx[k] < 0 || cam_idx[k] >= n_cams || pt_idx[k] < 0 || pt_idx[k] >= n_pts)
      return fail(BA_EINVAL, "observation index out of range");
  ba_problem* p = new (std::nothrow) ba_problem();
  if (!p) return fail(BA_EINVAL, "out of host memory");
  p->opt = o;
  std::string err;
  try {
    const std::vector<int32_t> ci = set_order(p, n_cams, n_pts, n_obs, cam_idx, pt_idx);
    err = ba::build_plan(n_cams, n_pts, n_obs, ci.data(), pt_idx, &p->plan);
  } catch (const std::bad_alloc&) {
    err = "out of host memory";
  }
  if (!err.empty()) {
    delete p;
    const bool unsup = err.find("at most") != std::string::npos;
    return fail(unsup ? BA_EUNSUPPORTED : BA_EINVAL, err);
  }
  return finish_create(p, out);
}

ba_status ba_pgo_create(const ba_options* opt, int32_t n_poses, int64_t n_edges, const int32_t* ei,
                        const int32_t* ej, ba_problem** out) {
  if (!out) return fail(BA_EINVAL, "out is null");
  *out = nullptr;
  if (!ei || !ej) return fail(BA_EINVAL, "edge arrays must not be null");
  if (n_poses <= 0 || n_edges <= 0) return fail(BA_EINVAL, "a pose graph needs poses and edges");
  if (n_edges > (int64_t)(INT32_MAX / 4)) return fail(BA_EUNSUPPORTED, "at most 2^29 edges");
  for (int64_t e = 0; e < n_edges; ++e) {
    if (ei[e] < 0 || ei[e] >= n_poses || ej[e] < 0 || ej[e] >= n_poses)
      return fail(BA_EINVAL, "edge endpoint out of range");
    if (ei[e] == ej[e]) return fail(BA_EINVAL, "an edge joins a pose to itself");
  }
  ba_options o;
  if (opt) o = *opt;
  else ba_default_options(&o);
  if (o.precond != BA_PRECOND_BLOCK_JACOBI || o.enable_backward || o.huber_delta > 0.0)
    return fail(BA_EUNSUPPORTED,
                "pose graphs take the squared loss, block-Jacobi preconditioning and no adjoint");
  o.cam_dof = 6;
  const ba_status st = check_options(o, n_poses);
  if (st != BA_OK) return st;
  ba_problem* p = new (std::nothrow) ba_problem();
  if (!p) return fail(BA_EINVAL, "out of host memory");
  p->opt = o;
  p->pgo = true;
  p->n_edges = n_edges;
  std::string err;
  try {
    // edge e as point e seen by its two poses: the plan's block pattern is
    // then the diagonal plus one block per joined pair of poses
    const int64_t no = 2 * n_edges;
    std::vector<int32_t> cidx(no), pidx(no);
    for (int64_t e = 0; e < n_edges; ++e) {
      cidx[2 * e] = ei[e];
      cidx[2 * e + 1] = ej[e];
      pidx[2 * e] = pidx[2 * e + 1] = (int32_t)e;
    }
    cidx = set_order(p, n_poses, (int32_t)n_edges, no, cidx.data(), pidx.data());
    std::vector<int32_t> ii(n_edges), jj(n_edges);
    for (int64_t e = 0; e < n_edges; ++e) {
      ii[e] = cidx[2 * e];
      jj[e] = cidx[2 * e + 1];
    }
    ei = ii.data();
    ej = jj.data();
    err = ba::build_plan(n_poses, (int32_t)n_edges, no, cidx.data(), pidx.data(), &p->plan);
    if (err.empty()) {
      ba::Plan& P = p->plan;
      // no points to eliminate: the Schur tables are not needed
      for (auto* v : {&P.pair_x, &P.pair_y, &P.slot_blk, &P.slot_pb, &P.slot_pe, &P.slot_lead, &P.stab,
                      &P.swptr})
        std::vector<int32_t>().swap(*v);
      P.n_pairs = 0;
      P.n_schur_wg = 0;
      p->pg_ei.assign(ei, ei + n_edges);
      p->pg_ej.assign(ej, ej + n_edges);
      // each block's edges in ascending edge order
      std::vector<int32_t> cnt(P.nnzb + 1, 0), blk(n_edges);
      for (int64_t e = 0; e < n_edges; ++e) {
        const int32_t a = std::min(ei[e], ej[e]), b = std::max(ei[e], ej[e]);
        const int32_t* rb = P.S_col.data() + P.S_ptr[a] + 1;
        const int32_t* re = P.S_col.data() + P.S_ptr[a + 1];
        const int32_t* it = std::lower_bound(rb, re, b);
        if (it == re || *it != b) throw std::logic_error("edge block missing from the plan");
        blk[e] = (int32_t)(it - P.S_col.data());
        cnt[P.S_ptr[ei[e]] + 1]++;
        cnt[P.S_ptr[ej[e]] + 1]++;
        cnt[blk[e] + 1]++;
      }
      p->pg_ptr.assign(P.nnzb + 1, 0);
      for (int64_t k = 0; k < P.nnzb; ++k) p->pg_ptr[k + 1] = p->pg_ptr[k] + cnt[k + 1];
      p->pg_code.assign(p->pg_ptr[P.nnzb], 0);
      std::vector<int32_t> fill(p->pg_ptr.begin(), p->pg_ptr.end() - 1);
      for (int64_t e = 0; e < n_edges; ++e) {
        p->pg_code[fill[P.S_ptr[ei[e]]]++] = (int32_t)(2 * e + 1);
        p->pg_code[fill[P.S_ptr[ej[e]]]++] = (int32_t)(2 * e);
        p->pg_code[fill[blk[e]]++] = (int32_t)(2 * e);
      }
    }
  } catch (const std::bad_alloc&) {
    err = "out of host memory";
  } catch (const std::logic_error& x) {
    err = x.what();
  }
  if (!err.empty()) {
    delete p;
    const bool unsup = err.find("at most") != std::string::npos;
    return fail(unsup ? BA_EUNSUPPORTED : BA_EINVAL, err);
  }
  return finish_create(p, out);
}

ba_status ba_problem_workspace_bytes(const ba_problem* p, size_t* bytes) {
  if (!p || !bytes) return fail(BA_EINVAL, "null argument");
  *bytes = p->ws_needed;
  return BA_OK;
}

ba_status ba_problem_nnzb(const ba_problem* p, int64_t* nnzb) {
  if (!p || !nnzb) return fail(BA_EINVAL, "null argument");
  *nnzb = p->plan.nnzb;
  return BA_OK;
}

namespace {

// Uploads the symbolic structure into workspace ws (device memory of at
// least p->ws_needed bytes, 256-byte aligned) and clears what must start at
// zero.  pinned: host staging from hipHostMalloc, else the handle's own
// members (the allocation-free binding).
ba_status bind_workspace(ba_problem* p, void* ws, size_t bytes, void* stream, bool pinned) {
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->workspace = ws;
  p->ws_bytes = bytes;
  size_t total = 0;
  carve(p, reinterpret_cast<char*>(ws), &total);
  const ba::Plan& P = p->plan;
  ba::Buffers& b = p->b;
  hipStream_t s = p->stream;
  HIPCHK(upload(b.o_cam, P.o_cam, s));
  HIPCHK(upload(b.o_pt, P.o_pt, s));
  HIPCHK(upload(b.pt_ptr, P.pt_ptr, s));
  HIPCHK(upload(b.chunk_ptr, P.chunk_ptr, s));
  HIPCHK(upload(b.chunk_pt, P.chunk_pt, s));
  HIPCHK(upload(b.long_chunk, P.long_chunk, s));
  HIPCHK(upload(b.cam_ptr, P.cam_ptr, s));
  HIPCHK(upload(b.cam_obs, P.cam_obs, s));
  HIPCHK(upload(b.S_ptr, P.S_ptr, s));
  HIPCHK(upload(b.S_col, P.S_col, s));
  HIPCHK(upload(b.T_ptr, P.T_ptr, s));
  HIPCHK(upload(b.T_blk, P.T_blk, s));
  HIPCHK(upload(b.T_src, P.T_src, s));
  HIPCHK(upload(b.pair_x, P.pair_x, s));
  HIPCHK(upload(b.pair_y, P.pair_y, s));
  HIPCHK(upload(b.slot_blk, P.slot_blk, s));
  HIPCHK(upload(b.slot_pb, P.slot_pb, s));
  HIPCHK(upload(b.slot_pe, P.slot_pe, s));
  HIPCHK(upload(b.slot_lead, P.slot_lead, s));
  HIPCHK(upload(b.blk_row, P.blk_row, s));
  HIPCHK(upload(b.stab, p->stab_units, s));
  HIPCHK(upload(b.swptr, P.swptr, s));
  HIPCHK(upload(b.pcg_row, P.pcg_row, s));
  HIPCHK(upload(b.item_ptr, P.item_ptr, s));
  HIPCHK(upload(b.item_e, P.item_e, s));
  HIPCHK(upload(b.item_code, P.item_code, s));
  HIPCHK(upload(b.ucol_ptr, P.ucol_ptr, s));
  HIPCHK(upload(b.ucol, P.ucol, s));
  HIPCHK(upload(b.srow, P.srow, s));
  HIPCHK(upload(b.sitem_ptr, P.sitem_ptr, s));
  HIPCHK(upload(b.sitem_col, P.sitem_col, s));
  HIPCHK(upload(b.blk_pos, P.blk_pos, s));
  HIPCHK(upload(b.vcol_ptr, P.vcol_ptr, s));
  HIPCHK(upload(b.vcol, P.vcol, s));
  HIPCHK(upload(b.vbase, P.vbase, s));
  HIPCHK(upload(b.in_ptr, P.in_ptr, s));
  HIPCHK(upload(b.in_off, P.in_off, s));
  HIPCHK(upload(b.src_ptr, P.src_ptr, s));
  HIPCHK(upload(b.src, P.src, s));
  HIPCHK(upload(b.o_orig, P.o_orig, s));
  if (p->opt.precond == BA_PRECOND_LEARNED) {
    HIPCHK(upload(b.nbr_ptr, P.nbr_ptr, s));
    HIPCHK(upload(b.nbr, P.nbr, s));
    HIPCHK(upload(b.nbr_blk, P.nbr_blk, s));
    HIPCHK(upload(b.nbr_rev, P.nbr_rev, s));
  }
  if (p->reordered) HIPCHK(upload(b.cam_perm, p->cam_perm, s));
  if (p->pgo) {
    HIPCHK(upload(b.pg_ei, p->pg_ei, s));
    HIPCHK(upload(b.pg_ej, p->pg_ej, s));
    HIPCHK(upload(b.pg_ptr, p->pg_ptr, s));
    HIPCHK(upload(b.pg_code, p->pg_code, s));
    // the poses' rows carry zero intrinsics
    for (int i = 0; i < 2; ++i) HIPCHK(hipMemsetAsync(b.cams[i], 0, sizeof(double) * 10 * P.nc, s));
  }
  HIPCHK(hipMemsetAsync(b.fixed, p->opt.cam_dof == 6 ? ba::FIXED_INTRINSICS : 0, P.nc, s));
  HIPCHK(hipMemsetAsync(b.gsync, 0, sizeof(ba::GridSync), s));
  if (pinned) {
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&p->hinfo), sizeof(ba_step_info), hipHostMallocDefault));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&p->hscal), sizeof(ba::DevScalars), hipHostMallocDefault));
  } else {
    p->hinfo = &p->hinfo_local;
    p->hscal = &p->hscal_local;
  }
  *p->hscal = ba::DevScalars{0.0, p->lambda, 0, 0};
  HIPCHK(hipMemcpyAsync(b.dev, p->hscal, sizeof(ba::DevScalars), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  const bool pipe = p->opt.cg_variant == BA_CG_PIPELINED;
  const int maxg = p->opt.precision == BA_MIXED
                       ? ba::pcg_max_grid<float>(P.pcg_resident, pipe, streamed(p))
                       : ba::pcg_max_grid<double>(P.pcg_resident, pipe, streamed(p));
  if (maxg <= 0) return fail(BA_EHIP, "cooperative occupancy query failed");
  p->pcg_grid = streamed(p) ? P.sgrid : P.pcg_grid;
  if (p->pcg_grid > maxg || p->pcg_grid > ba::MAX_BARRIER_GROUPS * ba::BARRIER_FANIN)
    return fail(BA_EUNSUPPORTED, "too many cameras for one co-resident PCG grid");
  p->adj_grid_ok = p->opt.enable_backward &&
                   P.pcg_grid <= ba::pcg_max_grid<double>(P.pcg_resident, false);
  p->bound = true;
  return BA_OK;
}

}  // namespace

ba_status ba_problem_bind(ba_problem* p, void* ws, size_t bytes, void* stream) {
  if (!p || !ws) return fail(BA_EINVAL, "null argument");
  if (bytes < p->ws_needed) return fail(BA_EINVAL, "workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(BA_EINVAL, "workspace not 256-byte aligned");
  if (p->bound) return fail(BA_ESTATE, "problem already bound");
  HIPCHK(hipGetDevice(&p->device));
  return bind_workspace(p, ws, bytes, stream, true);
}

ba_status ba_problem_bind_static(ba_problem* p, void* stream) {
  if (!p) return fail(BA_EINVAL, "null argument");
  if (p->bound) return fail(BA_ESTATE, "problem already bound");
  if (p->ws_needed > ba::STATIC_SCRATCH_BYTES) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "the problem needs %zu bytes of workspace; the static scratch holds %zu (use ba_problem_bind)",
                  p->ws_needed, ba::STATIC_SCRATCH_BYTES);
    return fail(BA_EINVAL, msg);
  }
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(BA_EUNSUPPORTED, "device ordinal beyond 63");
  void* scratch = nullptr;
  HIPCHK(ba::static_scratch(dev, &scratch));
  p->device = dev;
  p->static_ws = true;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    g_static_owner[dev] = p;
  }
  const ba_status st = bind_workspace(p, scratch, ba::STATIC_SCRATCH_BYTES, stream, false);
  if (st != BA_OK) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_owner[dev] == p) g_static_owner[dev] = nullptr;
    p->static_ws = false;
  }
  return st;
}

ba_status ba_set_observations(ba_problem* p, const double* xy, const double* w) {
  if (!p || !xy) return fail(BA_EINVAL, "null argument");
  if (p->pgo) return fail(BA_EINVAL, "a pose graph takes ba_pgo_set_edges");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  ba::ObsArgs a{p->plan.no, p->b.o_orig, xy, w, p->b.o_xy, p->b.o_w, p->b.dev};
  HIPCHK(ba::launch_set_observations(a, p->stream));
  HIPCHK(hipMemcpyAsync(p->hscal, p->b.dev, sizeof(ba::DevScalars), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  const int32_t err = p->hscal->error;
  if (err) {
    p->hscal->error = 0;
    HIPCHK(hipMemcpyAsync(p->b.dev, p->hscal, sizeof(ba::DevScalars), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    p->have_obs = false;
    return fail(BA_EINVAL, (err & ba::ERR_NONFINITE_OBS) ? "non-finite observation" : "observation weight <= 0");
  }
  p->have_obs = true;
  p->lin_valid = false;
  return BA_OK;
}

ba_status ba_set_fixed_cameras(ba_problem* p, const uint8_t* mask) {
  if (!p) return fail(BA_EINVAL, "null problem");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  const uint8_t base = p->opt.cam_dof == 6 ? ba::FIXED_INTRINSICS : 0;
  std::vector<uint8_t> m(p->plan.nc, base);
  if (mask)
    for (int32_t i = 0; i < p->plan.nc; ++i)
      m[p->reordered ? p->cam_perm[i] : i] = mask[i] ? ba::FIXED_CAMERA : base;
  HIPCHK(hipMemcpyAsync(p->b.fixed, m.data(), m.size(), hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->lin_valid = false;
  return BA_OK;
}

ba_status ba_set_params(ba_problem* p, const double* cams, const double* pts) {
  if (!p || !cams || !pts) return fail(BA_EINVAL, "null argument");
  if (p->pgo) return fail(BA_EINVAL, "a pose graph takes ba_pgo_set_poses");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  HIPCHK(copy_cameras(p, cams, 10, p->b.cams[p->cur], 10, 10, false));
  HIPCHK(hipMemcpyAsync(p->b.pts[p->cur], pts, sizeof(double) * 3 * p->plan.np,
                        hipMemcpyDeviceToDevice, p->stream));
  p->have_params = true;
  p->lin_valid = false;
  return BA_OK;
}

ba_status ba_get_params(const ba_problem* p, double* cams, double* pts) {
  if (!p) return fail(BA_EINVAL, "null problem");
  if (p->pgo) return fail(BA_EINVAL, "a pose graph takes ba_pgo_get_poses");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  if (!p->have_params) return fail(BA_ESTATE, "parameters are not set");
  if (cams) HIPCHK(copy_cameras(p, p->b.cams[p->cur], 10, cams, 10, 10, true));
  if (pts)
    HIPCHK(hipMemcpyAsync(pts, p->b.pts[p->cur], sizeof(double) * 3 * p->plan.np,
                          hipMemcpyDeviceToDevice, p->stream));
  return BA_OK;
}

ba_status ba_pgo_set_edges(ba_problem* p, const double* T, const double* omega) {
  if (!p || !T) return fail(BA_EINVAL, "null argument");
  if (!p->pgo) return fail(BA_EINVAL, "not a pose graph");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  ba::PgoEdgeArgs a{p->n_edges, T, omega, p->b.pg_T, p->b.pg_om, p->b.dev};
  HIPCHK(ba::launch_pgo_set_edges(a, p->stream));
  HIPCHK(hipMemcpyAsync(p->hscal, p->b.dev, sizeof(ba::DevScalars), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  const int32_t err = p->hscal->error;
  if (err) {
    p->hscal->error = 0;
    HIPCHK(hipMemcpyAsync(p->b.dev, p->hscal, sizeof(ba::DevScalars), hipMemcpyHostToDevice, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    p->have_obs = false;
    return fail(BA_EINVAL, (err & ba::ERR_NONFINITE_OBS)
                               ? "non-finite measurement or information matrix"
                               : "measurement quaternion not of unit norm, or information matrix not "
                                 "symmetric with a positive diagonal");
  }
  p->have_obs = true;
  p->lin_valid = false;
  return BA_OK;
}

ba_status ba_pgo_set_poses(ba_problem* p, const double* poses) {
  if (!p || !poses) return fail(BA_EINVAL, "null argument");
  if (!p->pgo) return fail(BA_EINVAL, "not a pose graph");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  HIPCHK(copy_cameras(p, poses, 7, p->b.cams[p->cur], 10, 7, false));
  p->have_params = true;
  p->lin_valid = false;
  return BA_OK;
}

ba_status ba_pgo_get_poses(const ba_problem* p, double* poses) {
  if (!p || !poses) return fail(BA_EINVAL, "null argument");
  if (!p->pgo) return fail(BA_EINVAL, "not a pose graph");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  if (!p->have_params) return fail(BA_ESTATE, "poses are not set");
  HIPCHK(copy_cameras(p, p->b.cams[p->cur], 10, poses, 7, 7, true));
  return BA_OK;
}

ba_status ba_set_lambda(ba_problem* p, double lambda) {
  if (!p || !(lambda > 0.0)) return fail(BA_EINVAL, "lambda must be positive");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  HIPCHK(hipMemcpyAsync(p->hscal, p->b.dev, sizeof(ba::DevScalars), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->hscal->lambda = lambda;
  HIPCHK(hipMemcpyAsync(p->b.dev, p->hscal, sizeof(ba::DevScalars), hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->lambda = lambda;
  return BA_OK;
}

ba_status ba_get_lambda(const ba_problem* p, double* lambda) {
  if (!p || !lambda) return fail(BA_EINVAL, "null argument");
  *lambda = p->lambda;
  return BA_OK;
}

ba_status ba_set_cg(ba_problem* p, double rtol, int32_t maxiter) {
  if (!p || !(rtol >= 0.0) || maxiter < 1) return fail(BA_EINVAL, "bad CG settings");
  if (maxiter > p->opt.cg_maxiter)
    return fail(BA_EINVAL, "maxiter exceeds the cg_maxiter the problem was created with");
  p->cg_rtol = rtol;
  p->cg_maxiter = maxiter;
  return BA_OK;
}

ba_status ba_lm_step(ba_problem* p, ba_step_info* info) {
  ba_status st = require_ready(p);
  if (st != BA_OK) return st;
  return p->opt.precision == BA_MIXED ? lm_step_impl<float>(p, info) : lm_step_impl<double>(p, info);
}

ba_status ba_solve(ba_problem* p, int32_t max_iters, double rel_tol, int32_t plateau_steps,
                   ba_step_info* infos, int32_t* iters_done) {
  ba_status st = require_ready(p);
  if (st != BA_OK) return st;
  if (max_iters < 0 || plateau_steps < 1) return fail(BA_EINVAL, "bad stopping rule");
  int32_t done = 0, flat = 0;
  ba_status ret = BA_OK;
  for (int32_t it = 0; it < max_iters; ++it) {
    ba_step_info info;
    st = ba_lm_step(p, &info);
    int32_t reason = BA_STOP_NONE;
    if (st != BA_OK) {
      ret = st;
      reason = BA_STOP_ERROR;
    } else {
      ++done;
      const double dec = info.accepted ? (info.cost_before - info.cost_after) / info.cost_before : 0.0;
      flat = dec < rel_tol ? flat + 1 : 0;
      if (!info.accepted && info.lambda_used >= p->opt.lambda_max) {
        ret = fail(BA_ENOTCONV, "damping reached lambda_max");
        reason = BA_STOP_LAMBDA_MAX;
      } else if (flat >= plateau_steps) {
        reason = BA_STOP_PLATEAU;
      } else if (info.grad_inf <= 1e-12 * (1.0 + info.cost_before)) {
        reason = BA_STOP_GRADIENT;
      } else if (it + 1 == max_iters) {
        reason = BA_STOP_MAX_ITERS;
      }
    }
    info.stop_reason = reason;
    if (infos) infos[it] = info;
    if (reason != BA_STOP_NONE) break;
  }
  if (iters_done) *iters_done = done;
  return ret;
}

ba_status ba_backward(ba_problem* p, const double* dL_dcams, const double* dL_dpts, double* dL_dobs,
                      double* dL_dw, ba_step_info* info) {
  using namespace ba;
  if (!p) return fail(BA_EINVAL, "null problem");
  if (p->opt.huber_delta > 0.0)
    return fail(BA_EUNSUPPORTED, "the adjoint is implemented for the squared loss only");
  ba_status st = require_ready(p);
  if (st != BA_OK) return st;
  if (!p->opt.enable_backward) return fail(BA_ESTATE, "create the problem with enable_backward set");
  if (!dL_dcams || !dL_dpts || !dL_dobs) return fail(BA_EINVAL, "null argument");
  if (!p->adj_grid_ok)
    return fail(BA_EUNSUPPORTED, "the FP64 PCG does not fit the co-resident grid of this problem");
  const Plan& P = p->plan;
  Buffers& b = p->b;
  hipStream_t s = p->stream;
  const int nchunk = (int)P.chunk_ptr.size() - 1;
  const int cur = p->cur;
  p->lin_valid = false;  // the linearisation buffers are reused below
  HIPCHK(hipMemsetAsync(b.adj_dev, 0, sizeof(DevScalars), s));
  HIPCHK(hipMemsetAsync(b.adj_info, 0, sizeof(ba_step_info), s));
  HIPCHK(hipMemsetAsync(b.diagU, 0, 9 * sizeof(double) * P.nc, s));  // no damping term
  if (p->reordered) {
    HIPCHK(copy_cameras(p, dL_dcams, 10, b.adj_gcam, 10, 10, false));
    dL_dcams = b.adj_gcam;
  }
  AdjTangentArgs ta{P.nc, b.fixed, b.cams[cur], dL_dcams, b.adj_gt};
  HIPCHK(launch_adj_tangent(ta, s));
  AdjObsArgs oa{P.no, b.o_cam, b.o_pt, b.fixed, b.o_xy, b.o_w, b.cams[cur], b.pts[cur],
                b.adjA, b.adjJ, b.r};
  HIPCHK(launch_adj_obs(oa, s));
  // the adjoint holds only where the gradient vanishes: check it first
  HIPCHK(hipMemsetAsync(b.adj_stat, 0, 2 * sizeof(double), s));
  AdjStatArgs ga0{P.nc, P.np, b.cam_ptr, b.cam_obs, b.pt_ptr, b.adjJ, b.r, b.o_w, b.adj_stat};
  HIPCHK(launch_adj_stationarity(ga0, s));
  double stat[2] = {0.0, 0.0};
  HIPCHK(hipMemcpyAsync(stat, b.adj_stat, sizeof stat, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (!(stat[0] <= p->opt.adjoint_grad_tol * stat[1])) {
    if (info) {
      *info = ba_step_info{};
      info->grad_inf = stat[0];
      info->status = BA_ENOTCONV;
    }
    char msg[160];
    std::snprintf(msg, sizeof msg,
                  "theta is not a stationary point: max |g| = %.3e > adjoint_grad_tol x %.3e", stat[0],
                  stat[1]);
    return fail(BA_ENOTCONV, msg);
  }
  AdjPointArgs pa{b.chunk_ptr, b.chunk_pt, b.pt_ptr, b.o_pt, b.adjA, b.Vinv, b.adjY, b.gsync,
                  &b.adj_dev->error};
  HIPCHK(launch_adj_points(pa, nchunk, long_chunks(p), s));
  AdjCameraArgs ca{b.cam_ptr, b.cam_obs, b.o_pt, b.fixed, b.adjA, b.adjY, dL_dpts, b.adj_gt,
                   b.adjU, b.bS};
  HIPCHK(launch_adj_camera(ca, P.nc, s));
  AdjSchurArgs sa{b.slot_blk, b.slot_pb, b.slot_pe, b.slot_lead, b.pair_x, b.pair_y, b.blk_row,
                  b.S_ptr, b.adjA, b.adjY, b.adjU, b.adjS, b.Sdiag};
  HIPCHK(launch_adj_schur(sa, P.n_schur_wg, s));
  // block-Jacobi factors of the undamped blocks (lambda = 0 in adj_dev)
  CamFinishArgs cf{b.Sdiag, b.diagU, p->opt.diag_min, p->opt.diag_max, b.Minv, b.adj_dev, nullptr,
                   nullptr, nullptr};
  HIPCHK(launch_camera_finish<double>(cf, P.nc, s));
  PcgArgs ga{P.nc, p->opt.cg_maxiter, p->opt.adjoint_rtol, b.S_ptr, b.T_ptr, b.pcg_row, b.item_ptr,
             b.item_e, b.item_code, b.ucol_ptr, b.ucol, b.adjS, b.Sdiag, b.Minv, b.bS, b.adj_vc,
             b.zring, b.partA, b.partB, b.adj_info, b.gsync, &b.adj_dev->error};
  HIPCHK(launch_pcg<double>(ga, P.pcg_grid, P.pcg_resident, false, s));
  AdjBackArgs bb{b.chunk_ptr, b.chunk_pt, b.pt_ptr, b.o_cam, b.o_pt, b.o_orig, b.adjA, b.adjJ,
                 b.r, b.o_w, b.Vinv, b.adj_vc, dL_dpts, b.adj_vp, dL_dobs, dL_dw};
  HIPCHK(launch_adj_backsub(bb, nchunk, long_chunks(p), s));
  HIPCHK(hipMemcpyAsync(p->hinfo, b.adj_info, sizeof(ba_step_info), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(p->hscal, b.adj_dev, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  ba_step_info out = *p->hinfo;
  out.grad_inf = stat[0];
  const int32_t err = p->hscal->error;
  st = BA_OK;
  if (err & ERR_BARRIER) st = fail(BA_EHIP, "the PCG grid barrier timed out");
  else if (err & ERR_POINT_BLOCK) st = fail(BA_ENUMERIC, "an exact point block is not positive definite");
  else if (err & ERR_CAMERA_BLOCK) st = fail(BA_ENUMERIC, "an exact camera block is not positive definite");
  else if (!(out.cg_rel_resid <= p->opt.adjoint_rtol))
    st = fail(BA_ENOTCONV, "the adjoint PCG did not reach adjoint_rtol");
  out.status = st;
  if (info) *info = out;
  return st;
}

int64_t ba_gnn_num_params(void) { return ba::GNN_NPARAM; }

ba_status ba_set_gnn_params(ba_problem* p, const float* params) {
  if (!p) return fail(BA_EINVAL, "null problem");
  if (p->opt.precond != BA_PRECOND_LEARNED)
    return fail(BA_ESTATE, "create the problem with precond = BA_PRECOND_LEARNED");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  if (!params) {
    p->gnn_ready = false;
    return BA_OK;
  }
  HIPCHK(hipMemcpyAsync(p->b.pc_params, params, sizeof(float) * ba::GNN_NPARAM,
                        hipMemcpyDeviceToDevice, p->stream));
  HIPCHK(ba::launch_gnn_weights_bf16(p->b.pc_params, p->b.pc_wbf16, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->gnn_ready = true;
  return BA_OK;
}

ba_status ba_get_state(const ba_problem* p, void* blob, size_t* bytes) {
  if (!p || !bytes) return fail(BA_EINVAL, "null argument");
  const size_t np = point_count(p);
  const size_t need = sizeof(double) * (4 + 10 * (size_t)p->plan.nc + 3 * np);
  if (!blob) {
    *bytes = need;
    return BA_OK;
  }
  if (*bytes < need) return fail(BA_EINVAL, "state buffer too small");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  if (!p->have_params) return fail(BA_ESTATE, "parameters are not set");
  double* d = reinterpret_cast<double*>(blob);
  d[0] = 1.0;  // format version
  d[1] = p->plan.nc;
  d[2] = (double)np;
  d[3] = p->lambda;
  std::vector<double> cams(10 * (size_t)p->plan.nc);
  HIPCHK(hipMemcpyAsync(cams.data(), p->b.cams[p->cur], sizeof(double) * cams.size(), hipMemcpyDeviceToHost,
                        p->stream));
  if (np)
    HIPCHK(hipMemcpyAsync(d + 4 + 10 * (size_t)p->plan.nc, p->b.pts[p->cur], sizeof(double) * 3 * np,
                          hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  rows_to_caller(p, cams.data(), d + 4, 10);
  *bytes = need;
  return BA_OK;
}

ba_status ba_set_state(ba_problem* p, const void* blob, size_t bytes) {
  if (!p || !blob) return fail(BA_EINVAL, "null argument");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  const size_t np = point_count(p);
  const size_t need = sizeof(double) * (4 + 10 * (size_t)p->plan.nc + 3 * np);
  const double* d = reinterpret_cast<const double*>(blob);
  if (bytes != need || d[0] != 1.0 || d[1] != p->plan.nc || d[2] != (double)np)
    return fail(BA_EINVAL, "state blob does not match this problem");
  std::vector<double> cams(10 * (size_t)p->plan.nc);
  for (size_t c = 0; c < (size_t)p->plan.nc; ++c)
    std::memcpy(cams.data() + 10 * (p->reordered ? (size_t)p->cam_perm[c] : c), d + 4 + 10 * c,
                10 * sizeof(double));
  HIPCHK(hipMemcpyAsync(p->b.cams[p->cur], cams.data(), sizeof(double) * cams.size(), hipMemcpyHostToDevice,
                        p->stream));
  if (np)
    HIPCHK(hipMemcpyAsync(p->b.pts[p->cur], d + 4 + 10 * (size_t)p->plan.nc, sizeof(double) * 3 * np,
                          hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  p->have_params = true;
  p->lin_valid = false;
  return ba_set_lambda(p, d[3]);
}

ba_status ba_export(const ba_problem* p, int32_t field, void* dst, size_t bytes) {
  if (!p || !dst) return fail(BA_EINVAL, "null argument");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  const ba::Plan& P = p->plan;
  const ba::Buffers& b = p->b;
  const size_t no = P.no, nc = P.nc, np = P.np, nnzb = P.nnzb;
  const bool mixed = p->opt.precision == BA_MIXED;
  auto need = [&](size_t n) { return bytes == n; };
  auto fetch = [&](const void* src, size_t n, std::vector<char>& h) -> hipError_t {
    h.resize(n);
    hipError_t e = hipMemcpyAsync(h.data(), src, n, hipMemcpyDeviceToHost, p->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(p->stream);
  };
  std::vector<char> h;
  double* out = reinterpret_cast<double*>(dst);
  if (p->pgo && (field == BA_X_RESIDUAL || field == BA_X_WEIGHT || field == BA_X_JC || field == BA_X_JP ||
                 field == BA_X_GRAD_P || field == BA_X_V || field == BA_X_DP || field == BA_X_ADJ_VC ||
                 field == BA_X_ADJ_VP))
    return fail(BA_EINVAL, "a pose graph has no observation or point fields");
  switch (field) {
    case BA_X_RESIDUAL:
    case BA_X_WEIGHT: {
      const bool res = field == BA_X_RESIDUAL;
      if (!need(no * sizeof(double) * (res ? 2 : 1))) return fail(BA_EINVAL, "size mismatch");
      if (res) {
        // (r_x, r_y) are the first two words of each observation's 8-word record
        h.resize(no * 2 * sizeof(double));
        HIPCHK(hipMemcpy2DAsync(h.data(), 2 * sizeof(double), b.rec, 8 * sizeof(double), 2 * sizeof(double), no,
                                hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
      } else {
        HIPCHK(fetch(b.w, no * sizeof(double), h));
      }
      const double* v = reinterpret_cast<const double*>(h.data());
      for (size_t x = 0; x < no; ++x) {
        const size_t k = P.o_orig[x];
        if (res) {
          out[2 * k] = v[2 * x];
          out[2 * k + 1] = v[2 * x + 1];
        } else {
          out[k] = v[x];
        }
      }
      return BA_OK;
    }
    case BA_X_JC:
    case BA_X_JP: {
      const bool jc = field == BA_X_JC;
      const size_t per = jc ? 18 : 6;
      if (!need(no * per * sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      HIPCHK(fetch(b.J, no * ba::NJ * elem_bytes(p), h));
      for (size_t x = 0; x < no; ++x) {
        const size_t k = P.o_orig[x];
        for (size_t q = 0; q < per; ++q) {
          const size_t src = x * ba::NJ + (jc ? 0 : 18) + q;
          out[k * per + q] = mixed ? (double)reinterpret_cast<const float*>(h.data())[src]
                                   : reinterpret_cast<const double*>(h.data())[src];
        }
      }
      return BA_OK;
    }
    case BA_X_COST: {
      if (!need(sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      HIPCHK(fetch(b.dev, sizeof(ba::DevScalars), h));
      out[0] = reinterpret_cast<const ba::DevScalars*>(h.data())->F;
      return BA_OK;
    }
    case BA_X_GRAD_C:
    case BA_X_BS:
    case BA_X_DC: {
      if (!need(nc * 9 * sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      const double* src = field == BA_X_GRAD_C ? b.gc : field == BA_X_BS ? b.bS : b.x;
      HIPCHK(fetch(src, bytes, h));
      rows_to_caller(p, reinterpret_cast<const double*>(h.data()), out, 9);
      return BA_OK;
    }
    case BA_X_GRAD_P:
    case BA_X_DP: {
      if (!need(np * 3 * sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      HIPCHK(hipMemcpyAsync(dst, field == BA_X_GRAD_P ? b.gp : b.dp, bytes, hipMemcpyDeviceToHost,
                            p->stream));
      HIPCHK(hipStreamSynchronize(p->stream));
      return BA_OK;
    }
    case BA_X_PRECOND: {
      if (!need(nc * 81 * sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      const bool learned = p->opt.precond == BA_PRECOND_LEARNED && p->gnn_ready;
      HIPCHK(fetch(learned ? b.pcMinvL : b.Minv, bytes, h));
      rows_to_caller(p, reinterpret_cast<const double*>(h.data()), out, 81);
      return BA_OK;
    }
    case BA_X_ADJ_VC:
    case BA_X_ADJ_VP: {
      if (!p->opt.enable_backward) return fail(BA_ESTATE, "backward buffers are not enabled");
      const bool vc = field == BA_X_ADJ_VC;
      if (!need((vc ? nc * 9 : np * 3) * sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      if (vc) {
        HIPCHK(fetch(b.adj_vc, bytes, h));
        rows_to_caller(p, reinterpret_cast<const double*>(h.data()), out, 9);
        return BA_OK;
      }
      HIPCHK(hipMemcpyAsync(dst, b.adj_vp, bytes, hipMemcpyDeviceToHost, p->stream));
      HIPCHK(hipStreamSynchronize(p->stream));
      return BA_OK;
    }
    case BA_X_V: {
      if (!need(np * 9 * sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      HIPCHK(fetch(b.V, np * 6 * sizeof(double), h));
      const double* v = reinterpret_cast<const double*>(h.data());
      static const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
      for (size_t j = 0; j < np; ++j)
        for (int q = 0; q < 9; ++q) out[9 * j + q] = v[6 * j + map[q]];
      return BA_OK;
    }
    case BA_X_S_PTR: {
      if (!need((nc + 1) * sizeof(int64_t))) return fail(BA_EINVAL, "size mismatch");
      int64_t* o = reinterpret_cast<int64_t*>(dst);
      for (size_t a = 0; a <= nc; ++a) o[a] = p->reordered ? p->x_ptr[a] : P.S_ptr[a];
      return BA_OK;
    }
    case BA_X_PLAN: {
      if (!need(4 * sizeof(int64_t))) return fail(BA_EINVAL, "size mismatch");
      int64_t* o = reinterpret_cast<int64_t*>(dst);
      o[0] = P.pcg_resident ? 0 : (streamed(p) ? 2 : 1);
      o[1] = streamed(p) ? P.sgrid : P.pcg_grid;
      o[2] = P.n_pairs;
      o[3] = P.n_schur_wg;
      return BA_OK;
    }
    case BA_X_S_COL: {
      if (!need(nnzb * sizeof(int32_t))) return fail(BA_EINVAL, "size mismatch");
      std::memcpy(dst, p->reordered ? p->x_col.data() : P.S_col.data(), bytes);
      return BA_OK;
    }
    case BA_X_S: {
      if (!need(nnzb * 81 * sizeof(double))) return fail(BA_EINVAL, "size mismatch");
      HIPCHK(fetch(b.S, nnzb * 81 * elem_bytes(p), h));
      for (size_t q = 0; q < nnzb * 81; ++q)
        out[q] = mixed ? (double)reinterpret_cast<const float*>(h.data())[q]
                       : reinterpret_cast<const double*>(h.data())[q];
      std::vector<char> hd;
      HIPCHK(fetch(b.Sdiag, nc * 81 * sizeof(double), hd));  // diagonal blocks are kept in FP64
      const double* d = reinterpret_cast<const double*>(hd.data());
      for (size_t a = 0; a < nc; ++a)
        std::memcpy(out + (size_t)P.S_ptr[a] * 81, d + a * 81, 81 * sizeof(double));
      if (p->reordered) {
        // internal blocks to the caller's pattern (a block whose caller row
        // comes after its column is the transpose of the stored one)
        const std::vector<double> in(out, out + nnzb * 81);
        for (size_t k = 0; k < nnzb; ++k) {
          const double* src = in.data() + (size_t)p->x_blk[k] * 81;
          double* o = out + k * 81;
          for (int r = 0; r < 9; ++r)
            for (int cc = 0; cc < 9; ++cc) o[9 * r + cc] = p->x_tr[k] ? src[9 * cc + r] : src[9 * r + cc];
        }
      }
      return BA_OK;
    }
    default:
      return fail(BA_EINVAL, "unknown field");
  }
}

ba_status ba_set_profiling(ba_problem* p, int32_t enable) {
  return ba_set_profiling_mask(p, enable ? (1u << BA_NUM_PHASES) - 1u : 0u);
}

ba_status ba_set_profiling_mask(ba_problem* p, uint32_t mask) {
  if (!p) return fail(BA_EINVAL, "null problem");
  if (!usable(p)) return fail(BA_ESTATE, not_bound_msg(p));
  const bool enable = mask != 0;
  if (enable && !p->ev[0][0]) {
    for (int i = 0; i < BA_NUM_PHASES; ++i)
      for (int k = 0; k < 2; ++k) HIPCHK(hipEventCreate(&p->ev[i][k]));
  }
  for (int i = 0; i < BA_NUM_PHASES; ++i) {
    p->phase_ms[i] = 0.0;
    p->phase_n[i] = 0;
    p->phase_used[i] = false;
  }
  p->profiling = enable;
  p->profile_mask = mask;
  return BA_OK;
}

ba_status ba_get_phase_times(const ba_problem* p, double* ms, int64_t* n_out, int32_t n) {
  if (!p || !ms || n < 0 || n > BA_NUM_PHASES) return fail(BA_EINVAL, "bad argument");
  for (int i = 0; i < n; ++i) {
    ms[i] = p->phase_ms[i];
    if (n_out) n_out[i] = p->phase_n[i];
  }
  return BA_OK;
}

ba_status ba_graph_create(const ba_problem* p, ba_graph** out) {
  if (!p || !out) return fail(BA_EINVAL, "null argument");
  *out = nullptr;
  if (p->opt.precond != BA_PRECOND_LEARNED)
    return fail(BA_ESTATE, "the problem was not created with BA_PRECOND_LEARNED");
  ba_graph* g = new (std::nothrow) ba_graph();
  if (!g) return fail(BA_EINVAL, "out of host memory");
  g->nc = p->plan.nc;
  g->nnzb = p->plan.nnzb;
  g->nbr_ptr = p->plan.nbr_ptr;
  g->nbr = p->plan.nbr;
  g->rev = p->plan.nbr_rev;
  graph_carve(g, nullptr, &g->ws_needed);
  *out = g;
  return BA_OK;
}

ba_status ba_graph_workspace_bytes(const ba_graph* g, size_t* bytes) {
  if (!g || !bytes) return fail(BA_EINVAL, "null argument");
  *bytes = g->ws_needed;
  return BA_OK;
}

ba_status ba_graph_bind(ba_graph* g, void* ws, size_t bytes, void* stream) {
  if (!g || !ws) return fail(BA_EINVAL, "null argument");
  if (g->bound) return fail(BA_ESTATE, "graph already bound");
  if (bytes < g->ws_needed) return fail(BA_EINVAL, "workspace too small");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(BA_EINVAL, "workspace not 256-byte aligned");
  g->stream = reinterpret_cast<hipStream_t>(stream);
  size_t total = 0;
  graph_carve(g, reinterpret_cast<char*>(ws), &total);
  HIPCHK(upload(const_cast<int32_t*>(g->dev.nbr_ptr), g->nbr_ptr, g->stream));
  HIPCHK(upload(const_cast<int32_t*>(g->dev.nbr), g->nbr, g->stream));
  HIPCHK(upload(const_cast<int32_t*>(g->dev.rev), g->rev, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  g->bound = true;
  return BA_OK;
}

ba_status ba_graph_build(ba_graph* g, ba_problem* p) {
  if (!g || !p) return fail(BA_EINVAL, "null argument");
  if (!g->bound) return fail(BA_ESTATE, "graph is not bound");
  if (p->opt.precond != BA_PRECOND_LEARNED || !usable(p))
    return fail(BA_ESTATE, "the problem is not bound with BA_PRECOND_LEARNED");
  if (p->plan.nc != g->nc || p->plan.nnzb != g->nnzb || p->plan.nbr != g->nbr)
    return fail(BA_EINVAL, "the graph was created for another camera pattern");
  if (!p->have_system) return fail(BA_ESTATE, "run ba_lm_step first (no reduced system yet)");
  const ba::Buffers& b = p->b;
  ba::PcFeatureArgs fa{g->nc, b.nbr_ptr, b.nbr, b.nbr_blk, b.S, b.pcLinv, g->dev.X, g->dev.E, g->dev.w,
                       nullptr, nullptr};
  HIPCHK(p->opt.precision == BA_MIXED ? ba::launch_pc_features<float>(fa, p->stream)
                                      : ba::launch_pc_features<double>(fa, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return BA_OK;
}

ba_status ba_gnn_loss_grad(ba_graph* g, const float* params, float* grad, double* loss) {
  if (!g || !params || !grad) return fail(BA_EINVAL, "null argument");
  if (!g->bound) return fail(BA_ESTATE, "graph is not bound");
  HIPCHK(ba::launch_gnn_forward(g->dev, params, g->stream));
  HIPCHK(ba::launch_gnn_output(g->dev, params, nullptr, nullptr, true, g->stream));
  HIPCHK(ba::launch_gnn_backward(g->dev, params, grad, g->stream));
  double h = 0.0;
  HIPCHK(hipMemcpyAsync(&h, g->dev.loss, sizeof(double), hipMemcpyDeviceToHost, g->stream));
  HIPCHK(hipStreamSynchronize(g->stream));
  if (loss) *loss = h;
  return BA_OK;
}

ba_status ba_gnn_adam(int64_t n, float* params, const float* grad, float* m, float* v, int32_t step,
                      float lr, float beta1, float beta2, float eps, float grad_scale, void* stream) {
  if (!params || !grad || !m || !v || n <= 0 || step < 1) return fail(BA_EINVAL, "bad argument");
  HIPCHK(ba::launch_gnn_adam(n, params, grad, m, v, step, lr, beta1, beta2, eps, grad_scale,
                             reinterpret_cast<hipStream_t>(stream)));
  return BA_OK;
}

void ba_graph_destroy(ba_graph* g) { delete g; }

void ba_problem_destroy(ba_problem* p) {
  if (!p) return;
  if (p->static_ws) {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (p->device >= 0 && p->device < 64 && g_static_owner[p->device] == p) g_static_owner[p->device] = nullptr;
  }
  for (int i = 0; i < BA_NUM_PHASES; ++i)
    for (int k = 0; k < 2; ++k)
      if (p->ev[i][k]) (void)hipEventDestroy(p->ev[i][k]);
  if (!p->static_ws) {
    if (p->hinfo) (void)hipHostFree(p->hinfo);
    if (p->hscal) (void)hipHostFree(p->hscal);
  }
  delete p;
}

}  // extern "C"
