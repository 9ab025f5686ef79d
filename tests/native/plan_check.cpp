// Host-only check of the symbolic analysis (no GPU): builds the plan of a
// scene given as binary index arrays and verifies the streamed-PCG
// decomposition it derives.  Prints "ok ..." and exits 0, or names the
// violated property and exits 1.
//
// usage: plan_check <prefix>   (reads <prefix>.hdr: int64 n_cams, n_pts,
//                               n_obs; <prefix>.cam, <prefix>.pt: int32)
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "ba_internal.h"

using namespace ba;

static bool read_file(const std::string& fn, void* dst, size_t bytes) {
  FILE* f = std::fopen(fn.c_str(), "rb");
  if (!f) return false;
  const size_t n = std::fread(dst, 1, bytes, f);
  std::fclose(f);
  return n == bytes;
}

#define CHECK(cond, what)                  \
  do {                                     \
    if (!(cond)) {                         \
      std::printf("violated: %s\n", what); \
      return 1;                            \
    }                                      \
  } while (0)

// largest |a - b| over the co-visible camera pairs (a, b) of a plan
static int32_t bandwidth(const Plan& p) {
  int32_t bw = 0;
  for (int32_t a = 0; a < p.nc; ++a)
    for (int32_t e = p.S_ptr[a]; e < p.S_ptr[a + 1]; ++e) bw = std::max(bw, p.S_col[e] - a);
  return bw;
}

// "order" mode: the camera renumbering is a permutation, keeps the block
// count, and prints the bandwidth before and after
static int check_order(const int64_t* h, const std::vector<int32_t>& cam, const std::vector<int32_t>& pt) {
  const int32_t nc = (int32_t)h[0];
  const std::vector<int32_t> ord = camera_order(nc, (int32_t)h[1], h[2], cam.data(), pt.data());
  CHECK((int32_t)ord.size() == nc, "one position per camera");
  std::vector<char> hit(nc, 0);
  for (int32_t c = 0; c < nc; ++c) {
    CHECK(ord[c] >= 0 && ord[c] < nc && !hit[ord[c]], "the order is a permutation");
    hit[ord[c]] = 1;
  }
  std::vector<int32_t> cam2(cam.size());
  for (size_t k = 0; k < cam.size(); ++k) cam2[k] = ord[cam[k]];
  Plan a, b;
  CHECK(build_plan(nc, (int32_t)h[1], h[2], cam.data(), pt.data(), &a).empty(), "plan in the given order");
  CHECK(build_plan(nc, (int32_t)h[1], h[2], cam2.data(), pt.data(), &b).empty(), "plan in the new order");
  CHECK(a.nnzb == b.nnzb && a.n_pairs == b.n_pairs, "renumbering keeps the blocks and pairs");
  std::printf("ok order %d %d\n", bandwidth(a), bandwidth(b));
  return 0;
}

int main(int argc, char** argv) {
  if (argc != 2 && argc != 3) return 2;
  const std::string pre = argv[1];
  int64_t h[3];
  if (!read_file(pre + ".hdr", h, sizeof h)) return 2;
  std::vector<int32_t> cam(h[2]), pt(h[2]);
  if (!read_file(pre + ".cam", cam.data(), 4 * h[2]) || !read_file(pre + ".pt", pt.data(), 4 * h[2])) return 2;
  if (argc == 3 && std::string(argv[2]) == "order") return check_order(h, cam, pt);
  Plan p;
  const std::string err = build_plan((int32_t)h[0], (int32_t)h[1], h[2], cam.data(), pt.data(), &p);
  if (!err.empty()) {
    std::printf("plan error: %s\n", err.c_str());
    return 1;
  }
  {
    // chunks: cover every position and point in order, none empty when it
    // has points with positions, at most CHUNK positions and CHUNK points
    // each, or one point seen more than CHUNK times (and then listed)
    const size_t nch = p.chunk_ptr.size() - 1;
    CHECK(p.chunk_ptr.size() == p.chunk_pt.size() && p.chunk_ptr.front() == 0 && p.chunk_pt.front() == 0 &&
              p.chunk_ptr.back() == h[2] && p.chunk_pt.back() == h[1],
          "chunks cover the positions and points");
    size_t nlong = 0;
    for (size_t c = 0; c < nch; ++c) {
      const int32_t x0 = p.chunk_ptr[c], x1 = p.chunk_ptr[c + 1], j0 = p.chunk_pt[c], j1 = p.chunk_pt[c + 1];
      CHECK(x0 <= x1 && j0 < j1, "chunks ascend and hold at least one point");
      CHECK(p.pt_ptr[j0] == x0 && p.pt_ptr[j1] == x1, "chunks are point-aligned");
      if (x1 - x0 > CHUNK) {
        CHECK(j1 - j0 == 1, "a chunk beyond CHUNK positions holds one point");
        CHECK(nlong < p.long_chunk.size() && p.long_chunk[nlong] == (int32_t)c, "long chunks listed in order");
        ++nlong;
      } else {
        CHECK(j1 - j0 <= CHUNK, "at most CHUNK points per chunk");
      }
    }
    CHECK(nlong == p.long_chunk.size(), "only long chunks listed");
  }
  if (p.pcg_resident) {
    CHECK(p.sgrid == 0 && p.srow.empty() && p.blk_pos.empty(), "resident plans carry no streamed decomposition");
    std::printf("ok resident\n");
    return 0;
  }
  if (p.sgrid == 0) {
    // too many block columns per workgroup for the streamed kernel: the
    // mixed solve reads the stored blocks per item instead
    CHECK(p.max_vcol > STREAM_COLS, "a streamed decomposition is dropped only beyond the column capacity");
    CHECK(p.srow.empty() && p.blk_pos.empty() && p.sitem_col.empty() && p.in_off.empty(),
          "no streamed arrays without a streamed decomposition");
    std::printf("ok unstreamed max_columns=%d\n", p.max_vcol);
    return 0;
  }
  const int32_t G = p.sgrid, nc = p.nc;
  CHECK(G >= 1 && G <= PCG_MAX_GRID, "streamed grid within the co-resident limit");
  CHECK(p.max_vcol <= STREAM_COLS, "columns within the streamed kernel's capacity");
  CHECK((int32_t)p.srow.size() == G + 1 && p.srow[0] == 0 && p.srow[G] == nc, "row ranges cover the cameras");
  std::vector<int32_t> owner(nc, -1);
  for (int32_t g = 0; g < G; ++g) {
    const int32_t nr = p.srow[g + 1] - p.srow[g];
    CHECK(nr >= 1 && nr <= STREAM_RMAX, "1..STREAM_RMAX rows per workgroup");
    for (int32_t a = p.srow[g]; a < p.srow[g + 1]; ++a) owner[a] = g;
  }
  // items: every upper off-diagonal block once, by its row's owner, in row order
  CHECK((int64_t)p.blk_pos.size() == p.nnzb, "one item slot per stored block");
  int64_t items = 0;
  for (int32_t g = 0; g < G; ++g) {
    int32_t it = p.sitem_ptr[g];
    const int32_t vb = p.vcol_ptr[g], nv = p.vcol_ptr[g + 1] - vb;
    CHECK(nv <= STREAM_COLS, "at most STREAM_COLS columns per workgroup");
    for (int32_t j = 1; j < nv; ++j) CHECK(p.vcol[vb + j - 1] < p.vcol[vb + j], "columns sorted and distinct");
    for (int32_t a = p.srow[g]; a < p.srow[g + 1]; ++a) {
      CHECK(p.blk_pos[p.S_ptr[a]] == -1, "diagonal blocks are not streamed");
      for (int32_t e = p.S_ptr[a] + 1; e < p.S_ptr[a + 1]; ++e, ++it) {
        CHECK(p.blk_pos[e] == it, "block -> item in row order");
        const int32_t j = p.sitem_col[it];
        CHECK(j >= 0 && j < nv && p.vcol[vb + j] == p.S_col[e], "item column");
      }
    }
    CHECK(it == p.sitem_ptr[g + 1], "item count per workgroup");
    items += p.sitem_ptr[g + 1] - p.sitem_ptr[g];
    CHECK(p.vbase[g] % 16 == 0, "exchange region starts on a 128-byte line");
    const int64_t end = p.vbase[g] + 9LL * nv;
    CHECK(end <= p.rstride && (g + 1 == G || end <= p.vbase[g + 1]), "exchange regions disjoint");
  }
  CHECK(items == p.nnzb - nc, "every upper off-diagonal block streamed once");
  CHECK(p.rstride % 16 == 0, "ring slot a whole number of lines");
  // received column sums: exactly the (sender, column) pairs of other
  // workgroups' columns in the receiver's rows, ascending sender, senders listed
  int64_t remote = 0;
  for (int32_t g = 0; g < G; ++g)
    for (int32_t j = p.vcol_ptr[g]; j < p.vcol_ptr[g + 1]; ++j) remote += owner[p.vcol[j]] != g;
  CHECK((int64_t)p.in_off.size() == remote && p.in_ptr[nc] == remote, "one received sum per remote column");
  for (int32_t b = 0; b < nc; ++b) {
    int32_t prev = -1;
    for (int32_t k = p.in_ptr[b]; k < p.in_ptr[b + 1]; ++k) {
      const int32_t off = p.in_off[k];
      const int32_t g = (int32_t)(std::upper_bound(p.vbase.begin(), p.vbase.end(), off) - p.vbase.begin()) - 1;
      CHECK(g >= 0 && g > prev && g != owner[b], "senders ascending, not the owner");
      CHECK((off - p.vbase[g]) % 9 == 0, "slot aligned to a column");
      const int32_t j = (off - p.vbase[g]) / 9;
      CHECK(j < p.vcol_ptr[g + 1] - p.vcol_ptr[g] && p.vcol[p.vcol_ptr[g] + j] == b, "slot holds the row's column");
      const int32_t o = owner[b];
      CHECK(std::find(p.src.begin() + p.src_ptr[o], p.src.begin() + p.src_ptr[o + 1], g) !=
                p.src.begin() + p.src_ptr[o + 1],
            "sender listed for the receiving workgroup");
      prev = g;
    }
  }
  int32_t max_in = 0, max_src = 0;
  for (int32_t g = 0; g < G; ++g) {
    max_in = std::max(max_in, p.in_ptr[p.srow[g + 1]] - p.in_ptr[p.srow[g]]);
    max_src = std::max(max_src, p.src_ptr[g + 1] - p.src_ptr[g]);
  }
  std::printf("ok streamed G=%d items=%lld remote=%lld max_in=%d max_senders=%d\n", G, (long long)items,
              (long long)remote, max_in, max_src);
  return 0;
}
