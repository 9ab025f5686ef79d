// Host-side symbolic analysis of the observation pattern.
//
// The sparsity of J, and hence of J^T J and of the reduced camera matrix,
// depends only on which camera sees which point, so it is analysed once per
// problem and reused by every LM iteration (the paper caches its symbolic
// sparse-product table the same way, Sec. IV-B-1).  Produces:
//   - observation "positions": the observations sorted by (point, camera,
//     original index), so every point's track is a contiguous, camera-sorted
//     run;
//   - point-aligned chunks of at most CHUNK positions and at most CHUNK
//     points (one workgroup each), or of one point seen more than CHUNK
//     times (listed in long_chunk);
//   - positions grouped by camera;
//   - the upper block pattern of the reduced camera matrix (camera a <= b
//     share a point), diagonal first in each row, plus its transpose lists;
//   - for every S block the list of observation pairs (x, y) feeding it (the
//     numeric Schur product's table), and the packing of the blocks' pair
//     chunks into workgroups of SCHUR_SLOTS chunk slots.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <numeric>

#include "ba_internal.h"

namespace ba {

// Reverse Cuthill-McKee order of the camera co-visibility graph (cameras
// adjacent when they share a point): each connected component from an
// unvisited camera of smallest degree, breadth first, every camera's
// unvisited neighbours in ascending degree (ties by index), the whole
// sequence reversed.  Blocks of the reduced matrix then lie near its
// diagonal, so a contiguous range of block rows touches few block columns
// and its column sums go to few other ranges.  order[c] = the position of
// camera c.
std::vector<int32_t> camera_order(int32_t nc, int32_t np, int64_t no, const int32_t* cidx,
                                  const int32_t* pidx) {
  // cameras of every point, then every camera's neighbours (both directions)
  std::vector<int64_t> pp(np + 1, 0);
  for (int64_t k = 0; k < no; ++k) pp[pidx[k] + 1]++;
  for (int32_t j = 0; j < np; ++j) pp[j + 1] += pp[j];
  std::vector<int32_t> pc(no);
  {
    std::vector<int64_t> fill(pp.begin(), pp.end() - 1);
    for (int64_t k = 0; k < no; ++k) pc[fill[pidx[k]]++] = cidx[k];
  }
  std::vector<std::vector<int32_t>> adj(nc);
  for (int32_t j = 0; j < np; ++j) {
    int32_t* b = pc.data() + pp[j];
    int32_t* e = pc.data() + pp[j + 1];
    std::sort(b, e);
    e = std::unique(b, e);
    for (int32_t* x = b; x < e; ++x)
      for (int32_t* y = x + 1; y < e; ++y) {
        adj[*x].push_back(*y);
        adj[*y].push_back(*x);
      }
  }
  std::vector<int32_t> deg(nc);
  for (int32_t c = 0; c < nc; ++c) {
    auto& v = adj[c];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    deg[c] = (int32_t)v.size();
  }
  std::vector<int32_t> by_deg(nc);
  std::iota(by_deg.begin(), by_deg.end(), 0);
  std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
  std::vector<char> seen(nc, 0);
  std::vector<int32_t> seq;
  seq.reserve(nc);
  std::vector<int32_t> nb;
  for (int32_t start : by_deg) {
    if (seen[start]) continue;
    size_t head = seq.size();
    seq.push_back(start);
    seen[start] = 1;
    while (head < seq.size()) {
      const int32_t u = seq[head++];
      nb.clear();
      for (int32_t v : adj[u])
        if (!seen[v]) {
          seen[v] = 1;
          nb.push_back(v);
        }
      std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
      seq.insert(seq.end(), nb.begin(), nb.end());
    }
  }
  std::vector<int32_t> order(nc);
  for (int32_t k = 0; k < nc; ++k) order[seq[nc - 1 - k]] = k;
  return order;
}

std::string build_plan(int32_t nc, int32_t np, int64_t no, const int32_t* cidx, const int32_t* pidx,
                       Plan* P) {
  char msg[256];
  if (nc <= 0 || np <= 0 || no <= 0) return "n_cams, n_pts and n_obs must be positive";
  if (no >= INT32_MAX / 2) return "n_obs too large for 32-bit positions";
  for (int64_t k = 0; k < no; ++k) {
    if (cidx[k] < 0 || cidx[k] >= nc || pidx[k] < 0 || pidx[k] >= np) {
      std::snprintf(msg, sizeof msg, "observation %lld has index out of range (cam %d, pt %d)",
                    (long long)k, cidx[k], pidx[k]);
      return msg;
    }
  }
  Plan& p = *P;
  p.nc = nc;
  p.np = np;
  p.no = no;

  // stable counting sort by camera, then by point: order (point, camera, k)
  std::vector<int64_t> by_cam(no), order(no);
  {
    std::vector<int64_t> cnt(nc + 1, 0);
    for (int64_t k = 0; k < no; ++k) cnt[cidx[k] + 1]++;
    for (int32_t i = 0; i < nc; ++i) cnt[i + 1] += cnt[i];
    for (int64_t k = 0; k < no; ++k) by_cam[cnt[cidx[k]]++] = k;
  }
  p.pt_ptr.assign(np + 1, 0);
  for (int64_t k = 0; k < no; ++k) p.pt_ptr[pidx[k] + 1]++;
  for (int32_t j = 0; j < np; ++j) p.pt_ptr[j + 1] += p.pt_ptr[j];
  {
    std::vector<int32_t> fill(p.pt_ptr.begin(), p.pt_ptr.end() - 1);
    for (int64_t i = 0; i < no; ++i) {
      const int64_t k = by_cam[i];
      order[fill[pidx[k]]++] = k;
    }
  }
  p.o_orig = order;
  p.o_cam.resize(no);
  p.o_pt.resize(no);
  for (int64_t x = 0; x < no; ++x) {
    p.o_cam[x] = cidx[order[x]];
    p.o_pt[x] = pidx[order[x]];
  }
  p.max_track = 0;
  for (int32_t j = 0; j < np; ++j) p.max_track = std::max(p.max_track, p.pt_ptr[j + 1] - p.pt_ptr[j]);

  // point-aligned chunks
  p.chunk_ptr.assign(1, 0);
  p.chunk_pt.assign(1, 0);
  {
    int32_t start = 0;
    for (int32_t j = 0; j < np; ++j) {
      // at most CHUNK positions and at most CHUNK points (unobserved points
      // have no positions) per chunk, except that a point seen more than
      // CHUNK times gets a chunk of its own
      if (j > p.chunk_pt.back() && (p.pt_ptr[j + 1] - start > CHUNK || j - p.chunk_pt.back() >= CHUNK)) {
        p.chunk_ptr.push_back(p.pt_ptr[j]);
        p.chunk_pt.push_back(j);
        start = p.pt_ptr[j];
      }
    }
    p.chunk_ptr.push_back((int32_t)no);
    p.chunk_pt.push_back(np);
    p.long_chunk.clear();
    for (size_t c = 0; c + 1 < p.chunk_ptr.size(); ++c)
      if (p.chunk_ptr[c + 1] - p.chunk_ptr[c] > CHUNK) p.long_chunk.push_back((int32_t)c);
  }

  // positions grouped by camera (ascending position inside a camera)
  p.cam_ptr.assign(nc + 1, 0);
  for (int64_t x = 0; x < no; ++x) p.cam_ptr[p.o_cam[x] + 1]++;
  for (int32_t i = 0; i < nc; ++i) p.cam_ptr[i + 1] += p.cam_ptr[i];
  p.cam_obs.resize(no);
  {
    std::vector<int32_t> fill(p.cam_ptr.begin(), p.cam_ptr.end() - 1);
    for (int64_t x = 0; x < no; ++x) p.cam_obs[fill[p.o_cam[x]]++] = (int32_t)x;
  }

  // track ranges with equal / larger camera
  std::vector<int32_t> same_lo(no), gt_lo(no);
  for (int32_t j = 0; j < np; ++j) {
    const int32_t lo = p.pt_ptr[j], hi = p.pt_ptr[j + 1];
    int32_t x = lo;
    while (x < hi) {
      int32_t y = x;
      while (y < hi && p.o_cam[y] == p.o_cam[x]) ++y;
      for (int32_t z = x; z < y; ++z) {
        same_lo[z] = x;
        gt_lo[z] = y;
      }
      x = y;
    }
  }

  // upper block pattern
  std::vector<std::vector<int32_t>> cols(nc);
  int64_t npairs = 0;
  for (int64_t x = 0; x < no; ++x) {
    const int32_t hi = p.pt_ptr[p.o_pt[x] + 1];
    npairs += hi - same_lo[x];
    for (int32_t y = gt_lo[x]; y < hi; ++y) cols[p.o_cam[x]].push_back(p.o_cam[y]);
  }
  if (npairs >= INT32_MAX) return "too many co-visible observation pairs";
  p.n_pairs = npairs;
  p.S_ptr.assign(nc + 1, 0);
  for (int32_t a = 0; a < nc; ++a) {
    auto& v = cols[a];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    p.S_ptr[a + 1] = p.S_ptr[a] + 1 + (int32_t)v.size();
  }
  p.nnzb = p.S_ptr[nc];
  p.S_col.resize(p.nnzb);
  p.blk_row.resize(p.nnzb);
  for (int32_t a = 0; a < nc; ++a)
    for (int32_t e = p.S_ptr[a]; e < p.S_ptr[a + 1]; ++e) p.blk_row[e] = a;
  for (int32_t a = 0; a < nc; ++a) {
    p.S_col[p.S_ptr[a]] = a;
    std::copy(cols[a].begin(), cols[a].end(), p.S_col.begin() + p.S_ptr[a] + 1);
  }

  // pair table grouped by block: diagonal pairs (same camera, y in
  // [same_lo, gt_lo), including y = x) and off-diagonal pairs (y in
  // [gt_lo, track end)); ascending x within a block
  std::vector<int32_t> pair_blk_of(npairs);
  std::vector<int32_t> bcount(p.nnzb + 1, 0);
  {
    int64_t q = 0;
    for (int64_t x = 0; x < no; ++x) {
      const int32_t a = p.o_cam[x];
      const int32_t hi = p.pt_ptr[p.o_pt[x] + 1];
      const int32_t* rb = p.S_col.data() + p.S_ptr[a] + 1;
      const int32_t* re = p.S_col.data() + p.S_ptr[a + 1];
      for (int32_t y = same_lo[x]; y < hi; ++y) {
        int32_t e = p.S_ptr[a];
        if (y >= gt_lo[x]) e = (int32_t)(std::lower_bound(rb, re, p.o_cam[y]) - p.S_col.data());
        pair_blk_of[q++] = e;
        bcount[e + 1]++;
      }
    }
  }
  for (int64_t e = 0; e < p.nnzb; ++e) bcount[e + 1] += bcount[e];
  p.pair_x.resize(npairs);
  p.pair_y.resize(npairs);
  {
    std::vector<int32_t> fill(bcount.begin(), bcount.end() - 1);
    int64_t q = 0;
    for (int64_t x = 0; x < no; ++x) {
      const int32_t hi = p.pt_ptr[p.o_pt[x] + 1];
      for (int32_t y = same_lo[x]; y < hi; ++y) {
        const int32_t e = pair_blk_of[q++];
        p.pair_x[fill[e]] = (int32_t)x;
        p.pair_y[fill[e]] = y;
        fill[e]++;
      }
    }
  }
  // chunks: a block of P pairs gets min(SCHUR_SLOTS, ceil(P / SCHUR_CHUNK))
  // chunks (at least one); blocks are packed into workgroups of SCHUR_SLOTS
  // slots next-fit in block order, so that a workgroup works on the blocks of
  // one or a few consecutive rows (shared observation data stays in cache)
  {
    std::vector<int32_t> nch(p.nnzb);
    std::vector<int32_t> order(p.nnzb);
    for (int64_t e = 0; e < p.nnzb; ++e) {
      const int32_t P = bcount[e + 1] - bcount[e];
      nch[e] = std::max(1, std::min(SCHUR_SLOTS, (P + SCHUR_CHUNK - 1) / SCHUR_CHUNK));
      order[e] = (int32_t)e;
    }
    p.slot_blk.clear();
    int32_t used = SCHUR_SLOTS;
    for (int32_t e : order) {
      if (used + nch[e] > SCHUR_SLOTS) {
        p.slot_blk.insert(p.slot_blk.end(), SCHUR_SLOTS, -1);
        p.slot_pb.insert(p.slot_pb.end(), SCHUR_SLOTS, 0);
        p.slot_pe.insert(p.slot_pe.end(), SCHUR_SLOTS, 0);
        p.slot_lead.insert(p.slot_lead.end(), SCHUR_SLOTS, 0);
        used = 0;
      }
      const size_t base = p.slot_blk.size() - SCHUR_SLOTS + used;
      const int32_t P = bcount[e + 1] - bcount[e], n = nch[e];
      for (int32_t k = 0; k < n; ++k) {
        p.slot_blk[base + k] = e;
        p.slot_pb[base + k] = bcount[e] + (int32_t)((int64_t)P * k / n);
        p.slot_pe[base + k] = bcount[e] + (int32_t)((int64_t)P * (k + 1) / n);
        p.slot_lead[base + k] = k == 0 ? n : 0;
      }
      used += n;
    }
    p.n_schur_wg = (int32_t)(p.slot_blk.size() / SCHUR_SLOTS);
    // wavefront steps: a wavefront takes as many steps as its longest chunk
    p.swptr.assign((size_t)p.n_schur_wg * SCHUR_WAVES + 1, 0);
    int64_t steps = 0;
    for (int32_t g = 0; g < p.n_schur_wg; ++g)
      for (int v = 0; v < SCHUR_WAVES; ++v) {
        int32_t n = 0;
        for (int s = 0; s < SCHUR_WAVE_SLOTS; ++s) {
          const size_t k = (size_t)g * SCHUR_SLOTS + v * SCHUR_WAVE_SLOTS + s;
          if (p.slot_blk[k] >= 0) n = std::max(n, p.slot_pe[k] - p.slot_pb[k]);
        }
        if (steps + n > INT32_MAX / SCHUR_ROWS) return "Schur step table too large";
        p.swptr[(size_t)g * SCHUR_WAVES + v] = (int32_t)steps;
        steps += n;
      }
    p.swptr.back() = (int32_t)steps;
    p.stab.assign((size_t)steps * SCHUR_ROWS, -1);
    for (int32_t g = 0; g < p.n_schur_wg; ++g)
      for (int v = 0; v < SCHUR_WAVES; ++v) {
        const size_t t0 = p.swptr[(size_t)g * SCHUR_WAVES + v];
        for (int s = 0; s < SCHUR_WAVE_SLOTS; ++s) {
          const size_t k = (size_t)g * SCHUR_SLOTS + v * SCHUR_WAVE_SLOTS + s;
          if (p.slot_blk[k] < 0) continue;
          for (int32_t i = p.slot_pb[k]; i < p.slot_pe[k]; ++i) {
            const size_t row = (t0 + (size_t)(i - p.slot_pb[k])) * SCHUR_ROWS;
            const int32_t x = p.pair_x[i], y = p.pair_y[i];
            p.stab[row + 2 * s] = x;
            p.stab[row + 2 * s + 1] = x == y ? -2 - x : y;
          }
        }
      }
  }

  // transpose lists: row b receives upper blocks (a, b) with a < b, ascending a
  p.T_ptr.assign(nc + 1, 0);
  for (int32_t a = 0; a < nc; ++a)
    for (int32_t e = p.S_ptr[a] + 1; e < p.S_ptr[a + 1]; ++e) p.T_ptr[p.S_col[e] + 1]++;
  for (int32_t b = 0; b < nc; ++b) p.T_ptr[b + 1] += p.T_ptr[b];
  p.T_blk.resize(p.T_ptr[nc]);
  p.T_src.resize(p.T_ptr[nc]);
  {
    std::vector<int32_t> fill(p.T_ptr.begin(), p.T_ptr.end() - 1);
    for (int32_t a = 0; a < nc; ++a)
      for (int32_t e = p.S_ptr[a] + 1; e < p.S_ptr[a + 1]; ++e) {
        const int32_t b = p.S_col[e];
        p.T_blk[fill[b]] = e;
        p.T_src[fill[b]] = a;
        fill[b]++;
      }
  }

  // camera co-visibility graph: for row i the off-diagonal upper blocks of
  // row i, then the blocks (a, i), a < i; rev[s] is the slot of the same
  // block seen from the other camera
  {
    p.nbr_ptr.assign(nc + 1, 0);
    for (int32_t i = 0; i < nc; ++i)
      p.nbr_ptr[i + 1] = p.nbr_ptr[i] + (p.S_ptr[i + 1] - p.S_ptr[i] - 1) + (p.T_ptr[i + 1] - p.T_ptr[i]);
    const int32_t ns = p.nbr_ptr[nc];
    p.nbr.resize(ns);
    p.nbr_blk.resize(ns);
    p.nbr_rev.resize(ns);
    std::vector<int32_t> up_slot(p.nnzb, -1), lo_slot(p.nnzb, -1);
    for (int32_t i = 0; i < nc; ++i) {
      int32_t s = p.nbr_ptr[i];
      for (int32_t e = p.S_ptr[i] + 1; e < p.S_ptr[i + 1]; ++e, ++s) {
        p.nbr[s] = p.S_col[e];
        p.nbr_blk[s] = e;
        up_slot[e] = s;
      }
      for (int32_t t = p.T_ptr[i]; t < p.T_ptr[i + 1]; ++t, ++s) {
        p.nbr[s] = p.T_src[t];
        p.nbr_blk[s] = p.T_blk[t];
        lo_slot[p.T_blk[t]] = s;
      }
    }
    for (int32_t s = 0; s < ns; ++s) {
      const int32_t e = p.nbr_blk[s];
      p.nbr_rev[s] = up_slot[e] == s ? lo_slot[e] : up_slot[e];
    }
  }

  // PCG workgroups: contiguous row ranges.  First try ranges of at most
  // PCG_IPG * PCG_GROUPS items (block values register-resident); if that
  // needs more than PCG_MAX_GRID workgroups, split the items evenly over
  // PCG_MAX_GRID workgroups and stream the block values.
  {
    std::vector<int64_t> row_items(nc);
    int64_t total = 0;
    for (int32_t a = 0; a < nc; ++a) {
      row_items[a] = (p.S_ptr[a + 1] - p.S_ptr[a]) + (p.T_ptr[a + 1] - p.T_ptr[a]);
      total += row_items[a];
    }
    auto partition = [&](int64_t cap, int64_t target, std::vector<int32_t>& rows) {
      rows.assign(1, 0);
      int64_t items = 0;
      int32_t nrow = 0;
      for (int32_t a = 0; a < nc; ++a) {
        if (cap > 0 && row_items[a] > cap) return false;
        const bool close = nrow > 0 && (nrow == PCG_RMAX || (cap > 0 && items + row_items[a] > cap) ||
                                        (target > 0 && items >= target));
        if (close) {
          rows.push_back(a);
          items = 0;
          nrow = 0;
        }
        items += row_items[a];
        ++nrow;
      }
      rows.push_back(nc);
      return true;
    };
    p.pcg_resident = partition((int64_t)PCG_IPG * PCG_GROUPS, 0, p.pcg_row) &&
                     (int32_t)p.pcg_row.size() - 1 <= PCG_MAX_GRID;
    if (!p.pcg_resident) partition(0, (total + PCG_MAX_GRID - 1) / PCG_MAX_GRID, p.pcg_row);
    p.pcg_grid = (int32_t)p.pcg_row.size() - 1;
    if (p.pcg_grid > PCG_MAX_GRID) {
      std::snprintf(msg, sizeof msg, "the reduced camera system needs %d PCG workgroups; at most %d",
                    p.pcg_grid, PCG_MAX_GRID);
      return msg;
    }
    p.item_ptr.assign(p.pcg_grid + 1, 0);
    p.ucol_ptr.assign(p.pcg_grid + 1, 0);
    p.item_e.clear();
    p.item_code.clear();
    p.ucol.clear();
    p.max_ucol = 0;
    std::vector<int32_t> uc;
    for (int32_t g = 0; g < p.pcg_grid; ++g) {
      const int32_t r0 = p.pcg_row[g], r1 = p.pcg_row[g + 1];
      uc.clear();
      for (int32_t a = r0; a < r1; ++a) {
        for (int32_t e = p.S_ptr[a]; e < p.S_ptr[a + 1]; ++e) uc.push_back(p.S_col[e]);
        for (int32_t t = p.T_ptr[a]; t < p.T_ptr[a + 1]; ++t) uc.push_back(p.T_src[t]);
      }
      std::sort(uc.begin(), uc.end());
      uc.erase(std::unique(uc.begin(), uc.end()), uc.end());
      p.max_ucol = std::max(p.max_ucol, (int32_t)uc.size());
      auto local = [&](int32_t c) {
        return (int32_t)(std::lower_bound(uc.begin(), uc.end(), c) - uc.begin());
      };
      for (int32_t a = r0; a < r1; ++a) {
        for (int32_t e = p.S_ptr[a]; e < p.S_ptr[a + 1]; ++e) {
          const bool diag = e == p.S_ptr[a];
          p.item_e.push_back(diag ? a : e);
          p.item_code.push_back(local(p.S_col[e]) | (diag ? ITEM_DIAG : 0));
        }
        for (int32_t t = p.T_ptr[a]; t < p.T_ptr[a + 1]; ++t) {
          p.item_e.push_back(p.T_blk[t]);
          p.item_code.push_back(local(p.T_src[t]) | ITEM_TRANS);
        }
      }
      p.item_ptr[g + 1] = (int32_t)p.item_e.size();
      p.ucol.insert(p.ucol.end(), uc.begin(), uc.end());
      p.ucol_ptr[g + 1] = (int32_t)p.ucol.size();
    }
    if (p.max_ucol > PCG_ZCOLS) {
      std::snprintf(msg, sizeof msg,
                    "a PCG workgroup would read %d block columns; at most %d are supported",
                    p.max_ucol, PCG_ZCOLS);
      return msg;
    }
  }

  // Streamed plans: a decomposition of their own.  Each upper block is read
  // once per product, by the owner of its row, so rows are weighted by their
  // upper blocks (64 each) plus the column sums they receive (at most one per
  // lower block); contiguous ranges of at most STREAM_RMAX rows, at most
  // PCG_MAX_GRID of them, with the smallest largest weight (bisection on the
  // cap of a greedy split).
  p.srow.clear();
  p.sitem_ptr.clear();
  p.sitem_col.clear();
  p.blk_pos.clear();
  p.vcol_ptr.clear();
  p.vcol.clear();
  p.vbase.clear();
  p.in_ptr.clear();
  p.in_off.clear();
  p.src_ptr.clear();
  p.src.clear();
  p.rstride = 0;
  p.sgrid = 0;
  p.max_vcol = 0;
  if (!p.pcg_resident) {
    std::vector<int64_t> wgt(nc);
    int64_t total = 0, wmax = 0;
    for (int32_t a = 0; a < nc; ++a) {
      wgt[a] = 64 * (int64_t)(p.S_ptr[a + 1] - p.S_ptr[a]) + (p.T_ptr[a + 1] - p.T_ptr[a]);
      total += wgt[a];
      wmax = std::max(wmax, wgt[a]);
    }
    auto split = [&](int64_t cap, std::vector<int32_t>& rows) {
      rows.assign(1, 0);
      int64_t items = 0;
      int32_t nrow = 0;
      for (int32_t a = 0; a < nc; ++a) {
        if (nrow > 0 && (nrow == STREAM_RMAX || items + wgt[a] > cap)) {
          rows.push_back(a);
          items = 0;
          nrow = 0;
        }
        items += wgt[a];
        ++nrow;
      }
      rows.push_back(nc);
      return (int32_t)rows.size() - 1;
    };
    int64_t lo = wmax, hi = total;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (split(mid, p.srow) <= PCG_MAX_GRID)
        hi = mid;
      else
        lo = mid + 1;
    }
    if (split(lo, p.srow) > PCG_MAX_GRID) {
      std::snprintf(msg, sizeof msg, "the streamed PCG needs more than %d workgroups", PCG_MAX_GRID);
      return msg;
    }
    const int32_t G = p.sgrid = (int32_t)p.srow.size() - 1;
    p.sitem_ptr.assign(G + 1, 0);
    p.vcol_ptr.assign(G + 1, 0);
    p.vbase.assign(G, 0);
    p.blk_pos.assign((size_t)p.nnzb, -1);
    int64_t off = 0;
    std::vector<int32_t> vc;
    for (int32_t g = 0; g < G; ++g) {
      const int32_t r0 = p.srow[g], r1 = p.srow[g + 1];
      vc.clear();
      for (int32_t a = r0; a < r1; ++a)
        for (int32_t e = p.S_ptr[a] + 1; e < p.S_ptr[a + 1]; ++e) vc.push_back(p.S_col[e]);
      std::sort(vc.begin(), vc.end());
      vc.erase(std::unique(vc.begin(), vc.end()), vc.end());
      p.max_vcol = std::max(p.max_vcol, (int32_t)vc.size());
      for (int32_t a = r0; a < r1; ++a)
        for (int32_t e = p.S_ptr[a] + 1; e < p.S_ptr[a + 1]; ++e) {
          p.blk_pos[e] = (int32_t)p.sitem_col.size();
          p.sitem_col.push_back(
              (int32_t)(std::lower_bound(vc.begin(), vc.end(), p.S_col[e]) - vc.begin()));
        }
      p.sitem_ptr[g + 1] = (int32_t)p.sitem_col.size();
      off = (off + 15) & ~(int64_t)15;
      p.vbase[g] = (int32_t)std::min<int64_t>(off, INT32_MAX);
      off += 9 * (int64_t)vc.size();
      p.vcol.insert(p.vcol.end(), vc.begin(), vc.end());
      p.vcol_ptr[g + 1] = (int32_t)p.vcol.size();
    }
    p.rstride = (off + 15) & ~(int64_t)15;
  }
  if (!p.pcg_resident && (p.max_vcol > STREAM_COLS || p.rstride > INT32_MAX)) {
    // beyond the streamed kernel's LDS column capacity: no streamed
    // decomposition (the mixed solve then reads the stored blocks per item)
    const int32_t mv = p.max_vcol;
    for (auto* v : {&p.srow, &p.sitem_ptr, &p.sitem_col, &p.blk_pos, &p.vcol_ptr, &p.vcol, &p.vbase})
      v->clear();
    p.rstride = 0;
    p.sgrid = 0;
    p.max_vcol = mv;
  }
  if (p.sgrid > 0) {
    const int32_t G = p.sgrid;
    std::vector<int32_t> owner(nc);
    for (int32_t g = 0; g < G; ++g)
      for (int32_t a = p.srow[g]; a < p.srow[g + 1]; ++a) owner[a] = g;
    // incoming slots of every row, ascending sending workgroup; the senders
    // of every workgroup
    p.in_ptr.assign(nc + 1, 0);
    for (int32_t g = 0; g < G; ++g)
      for (int32_t j = p.vcol_ptr[g]; j < p.vcol_ptr[g + 1]; ++j)
        if (owner[p.vcol[j]] != g) p.in_ptr[p.vcol[j] + 1]++;
    for (int32_t b = 0; b < nc; ++b) p.in_ptr[b + 1] += p.in_ptr[b];
    p.in_off.resize(p.in_ptr[nc]);
    std::vector<int32_t> fill(p.in_ptr.begin(), p.in_ptr.end() - 1);
    std::vector<std::vector<int32_t>> senders(G);
    for (int32_t g = 0; g < G; ++g)
      for (int32_t j = p.vcol_ptr[g]; j < p.vcol_ptr[g + 1]; ++j) {
        const int32_t b = p.vcol[j], o = owner[b];
        if (o == g) continue;
        p.in_off[fill[b]++] = p.vbase[g] + 9 * (j - p.vcol_ptr[g]);
        if (senders[o].empty() || senders[o].back() != g) senders[o].push_back(g);
      }
    p.src_ptr.assign(G + 1, 0);
    for (int32_t g = 0; g < G; ++g) {
      p.src.insert(p.src.end(), senders[g].begin(), senders[g].end());
      p.src_ptr[g + 1] = (int32_t)p.src.size();
    }
  }
  return std::string();
}

}  // namespace ba
