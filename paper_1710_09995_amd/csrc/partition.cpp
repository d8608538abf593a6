// Block split and regroup for load balance (Section 3.2.1): the pre-processing
// that cuts the blocks of a multi-block grid into pieces, rewrites the
// connection and boundary tables for the pieces, and deals the pieces into
// balanced groups (one per device).  Host code only: no device is touched.
// The rules are stated with the declarations in include/cfd.h.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cfd.h"
#include "host_services.hpp"

namespace {

using cfd::host_fail;

struct Box {
  int32_t parent;
  int32_t lo[3];
  int32_t n[3];
};

// A half-open rectangle in the two transverse directions of a face.
struct Rect {
  int32_t lo[2], hi[2];
};

int64_t volume(const Box& b) { return (int64_t)b.n[0] * b.n[1] * b.n[2]; }

int extent(const cfd_dims& d, int a) { return a == 0 ? d.ni : a == 1 ? d.nj : d.nk; }

// The direction a box is cut across: its longest extent, equal extents going
// to the higher direction (i is the wavefront direction of the stage kernels).
int cut_direction(const Box& b) {
  int d = 2;
  if (b.n[1] > b.n[d]) d = 1;
  if (b.n[0] > b.n[d]) d = 0;
  return d;
}

void transverse(int d, int& t1, int& t2) {
  t1 = d == 0 ? 1 : 0;
  t2 = d == 2 ? 1 : 2;
}

// The box's cells on a d-face, in its parent's transverse indices.
Rect face_rect(const Box& b, int d) {
  int t1, t2;
  transverse(d, t1, t2);
  return Rect{{b.lo[t1], b.lo[t2]}, {b.lo[t1] + b.n[t1], b.lo[t2] + b.n[t2]}};
}

bool clip(Rect& r, const Rect& by) {
  for (int a = 0; a < 2; ++a) {
    r.lo[a] = std::max(r.lo[a], by.lo[a]);
    r.hi[a] = std::min(r.hi[a], by.hi[a]);
    if (r.lo[a] >= r.hi[a]) return false;
  }
  return true;
}

Rect moved(const Rect& r, const int32_t off[2]) {
  return Rect{{r.lo[0] + off[0], r.lo[1] + off[1]}, {r.hi[0] + off[0], r.hi[1] + off[1]}};
}

// Cells of the lower part when n cells are cut: the multiple of `align`
// nearest n/2 (equal distance: the lower), if it lies in [n/4, 3n/4] and leaves
// both parts min_width cells; else floor(n/2).
int cut_at(int n32, int align32, int min_width32) {
  const int64_t n = n32, align = align32, min_width = min_width32;   // 64-bit: no overflow near 2^31
  const int64_t below = n / (2 * align) * align;
  const int64_t above = below + align;
  const int64_t c = (n - 2 * below <= 2 * above - n) ? below : above;
  if (c > 0 && 4 * c >= n && 4 * c <= 3 * n && c >= min_width && n - c >= min_width) return (int)c;
  return n32 / 2;
}

std::vector<Box> make_plan(int nblk, const cfd_dims* dims, int64_t max_cells, int min_width, const int align[3]) {
  std::vector<Box> out, todo;
  for (int b = 0; b < nblk; ++b) {
    todo.push_back(Box{b, {0, 0, 0}, {dims[b].ni, dims[b].nj, dims[b].nk}});
    while (!todo.empty()) {     // depth first, the lower part first
      const Box x = todo.back();
      todo.pop_back();
      const int d = cut_direction(x);
      if (volume(x) > max_cells && x.n[d] >= 2 * (int64_t)min_width) {
        Box lower = x, upper = x;
        lower.n[d] = cut_at(x.n[d], align[d], min_width);
        upper.n[d] = x.n[d] - lower.n[d];
        upper.lo[d] = x.lo[d] + lower.n[d];
        todo.push_back(upper);
        todo.push_back(lower);
      } else {
        out.push_back(x);
      }
    }
  }
  return out;
}

void check_pieces(int nblk, const cfd_dims* dims, const cfd_piece* pieces, int npieces) {
  if (npieces <= 0 || !pieces) host_fail(CFD_EINVAL, "need at least one piece");
  std::vector<int64_t> covered(nblk, 0);
  for (int p = 0; p < npieces; ++p) {
    const cfd_piece& q = pieces[p];
    if (q.parent < 0 || q.parent >= nblk) host_fail(CFD_EINVAL, "piece " + std::to_string(p) + ": bad parent");
    for (int a = 0; a < 3; ++a)
      if (q.lo[a] < 0 || q.n[a] < 1 || q.lo[a] + q.n[a] > extent(dims[q.parent], a))
        host_fail(CFD_EINVAL, "piece " + std::to_string(p) + " lies outside its parent");
    covered[q.parent] += (int64_t)q.n[0] * q.n[1] * q.n[2];
  }
  // Every cell once: the volumes add up and no two pieces of a parent overlap
  // (pairwise, so O(pieces^2) per block: meant for up to some thousands).
  for (int b = 0; b < nblk; ++b)
    if (covered[b] != (int64_t)dims[b].ni * dims[b].nj * dims[b].nk)
      host_fail(CFD_EINVAL, "the pieces of block " + std::to_string(b) + " do not tile it");
  for (int p = 0; p < npieces; ++p)
    for (int r = p + 1; r < npieces; ++r) {
      const cfd_piece &a = pieces[p], &b = pieces[r];
      if (a.parent != b.parent) continue;
      bool apart = false;
      for (int x = 0; x < 3; ++x)
        apart = apart || a.lo[x] + a.n[x] <= b.lo[x] || b.lo[x] + b.n[x] <= a.lo[x];
      if (!apart) host_fail(CFD_EINVAL, "pieces " + std::to_string(p) + " and " + std::to_string(r) + " overlap");
    }
}

struct Tables {
  std::vector<cfd_conn> conns;
  std::vector<cfd_bc> bcs;
};

Tables make_tables(int nblk, const cfd_dims* dims, const cfd_conn* conns, int nconn, const cfd_bc* bcs, int nbc,
                   const std::vector<Box>& P) {
  // pieces that lie on each face of each parent, in piece order
  std::vector<std::vector<int>> on_face((size_t)nblk * 6);
  // pieces by (parent, direction, lower index in that direction)
  std::map<std::tuple<int, int, int>, std::vector<int>> starting_at;
  for (int q = 0; q < (int)P.size(); ++q) {
    const Box& x = P[q];
    for (int d = 0; d < 3; ++d) {
      if (x.lo[d] == 0) on_face[(size_t)x.parent * 6 + 2 * d].push_back(q);
      if (x.lo[d] + x.n[d] == extent(dims[x.parent], d)) on_face[(size_t)x.parent * 6 + 2 * d + 1].push_back(q);
      starting_at[{x.parent, d, x.lo[d]}].push_back(q);
    }
  }
  Tables T;
  for (int i = 0; i < nbc; ++i) {
    const cfd_bc& B = bcs[i];
    const int d = B.face >> 1;
    for (int q : on_face[(size_t)B.blk * 6 + B.face]) {
      const Rect own = face_rect(P[q], d);
      Rect r{{B.lo[0], B.lo[1]}, {B.hi[0], B.hi[1]}};
      if (!clip(r, own)) continue;
      cfd_bc o = B;
      o.blk = q;
      for (int a = 0; a < 2; ++a) {
        o.lo[a] = r.lo[a] - own.lo[a];
        o.hi[a] = r.hi[a] - own.lo[a];
      }
      T.bcs.push_back(o);
    }
  }
  for (int i = 0; i < nconn; ++i) {
    const cfd_conn& Cn = conns[i];
    const int d = Cn.face >> 1;
    const int32_t to_nbr[2] = {Cn.nbr_lo[0] - Cn.lo[0], Cn.nbr_lo[1] - Cn.lo[1]};
    const int32_t from_nbr[2] = {-to_nbr[0], -to_nbr[1]};
    for (int q : on_face[(size_t)Cn.blk * 6 + Cn.face]) {
      const Rect own = face_rect(P[q], d);
      Rect r{{Cn.lo[0], Cn.lo[1]}, {Cn.hi[0], Cn.hi[1]}};
      if (!clip(r, own)) continue;
      for (int s : on_face[(size_t)Cn.nbr * 6 + Cn.nbr_face]) {
        const Rect theirs = face_rect(P[s], d);
        Rect m = moved(r, to_nbr);          // in the neighbour parent's indices
        if (!clip(m, theirs)) continue;
        const Rect back = moved(m, from_nbr);
        cfd_conn o = Cn;
        o.blk = q;
        o.nbr = s;
        for (int a = 0; a < 2; ++a) {
          o.lo[a] = back.lo[a] - own.lo[a];
          o.hi[a] = back.hi[a] - own.lo[a];
          o.nbr_lo[a] = m.lo[a] - theirs.lo[a];
        }
        T.conns.push_back(o);
      }
    }
  }
  // seams inside a parent: the upper d-face of q against every piece that
  // starts where q ends, both sides listed
  for (int q = 0; q < (int)P.size(); ++q) {
    const Box& x = P[q];
    for (int d = 0; d < 3; ++d) {
      const int top = x.lo[d] + x.n[d];
      if (top == extent(dims[x.parent], d)) continue;
      auto it = starting_at.find({x.parent, d, top});
      if (it == starting_at.end()) continue;
      const Rect mine = face_rect(x, d);
      for (int s : it->second) {
        const Rect other = face_rect(P[s], d);
        Rect r = mine;
        if (!clip(r, other)) continue;
        cfd_conn up{}, down{};
        up.blk = q, up.face = 2 * d + 1, up.nbr = s, up.nbr_face = 2 * d;
        down.blk = s, down.face = 2 * d, down.nbr = q, down.nbr_face = 2 * d + 1;
        for (int a = 0; a < 2; ++a) {
          up.lo[a] = r.lo[a] - mine.lo[a];
          up.hi[a] = r.hi[a] - mine.lo[a];
          up.nbr_lo[a] = r.lo[a] - other.lo[a];
          down.lo[a] = r.lo[a] - other.lo[a];
          down.hi[a] = r.hi[a] - other.lo[a];
          down.nbr_lo[a] = r.lo[a] - mine.lo[a];
        }
        T.conns.push_back(up);
        T.conns.push_back(down);
      }
    }
  }
  return T;
}

// Writes n items to out (capacity cap); out == NULL asks for the count only.
template <typename T>
void deliver(const std::vector<T>& v, T* out, int32_t cap, int32_t* count, const char* what) {
  if (!count) host_fail(CFD_EINVAL, std::string("NULL count for ") + what);
  if (v.size() > (size_t)INT32_MAX) host_fail(CFD_EINVAL, std::string("too many ") + what);
  *count = (int32_t)v.size();
  if (!out) return;
  if (cap < (int32_t)v.size())
    host_fail(CFD_ENOMEM, std::string(what) + ": the output array holds " + std::to_string(cap) + ", " +
                              std::to_string(v.size()) + " needed");
  std::copy(v.begin(), v.end(), out);
}

}  // namespace

extern "C" {

cfd_status cfd_split_plan(int32_t nblk, const cfd_dims* dims, int64_t max_cells, int32_t min_width,
                          const int32_t align[3], cfd_piece* pieces, int32_t capacity, int32_t* npieces) {
  return cfd::host_guarded([&] {
    cfd::host_check_dims(nblk, dims);
    if (max_cells < 1) host_fail(CFD_EINVAL, "max_cells must be positive");
    if (min_width < 2) host_fail(CFD_EINVAL, "min_width must be at least the ghost depth (2)");
    int al[3] = {1, 1, 1};
    for (int a = 0; a < 3 && align; ++a) {
      if (align[a] < 1 || align[a] > (1 << 20)) host_fail(CFD_EINVAL, "align must be in [1, 2^20]");
      al[a] = align[a];
    }
    const std::vector<Box> P = make_plan(nblk, dims, max_cells, min_width, al);
    std::vector<cfd_piece> out(P.size());
    for (size_t q = 0; q < P.size(); ++q) {
      out[q].parent = P[q].parent;
      for (int a = 0; a < 3; ++a) {
        out[q].lo[a] = P[q].lo[a];
        out[q].n[a] = P[q].n[a];
      }
    }
    deliver(out, pieces, capacity, npieces, "pieces");
  });
}

cfd_status cfd_split_tables(int32_t nblk, const cfd_dims* dims, const cfd_conn* conns, int32_t nconn,
                            const cfd_bc* bcs, int32_t nbc, const cfd_piece* pieces, int32_t npieces,
                            cfd_conn* out_conns, int32_t conn_capacity, int32_t* nconn_out, cfd_bc* out_bcs,
                            int32_t bc_capacity, int32_t* nbc_out) {
  return cfd::host_guarded([&] {
    cfd::host_check_case(nblk, dims, nconn, conns, nbc, bcs);
    check_pieces(nblk, dims, pieces, npieces);
    std::vector<Box> P(npieces);
    for (int q = 0; q < npieces; ++q) {
      P[q].parent = pieces[q].parent;
      for (int a = 0; a < 3; ++a) {
        P[q].lo[a] = pieces[q].lo[a];
        P[q].n[a] = pieces[q].n[a];
      }
    }
    const Tables T = make_tables(nblk, dims, conns, nconn, bcs, nbc, P);
    // both counts are set before either array is checked, so one call with
    // NULL arrays sizes both
    if (!nconn_out || !nbc_out) host_fail(CFD_EINVAL, "NULL count");
    *nconn_out = (int32_t)T.conns.size();
    *nbc_out = (int32_t)T.bcs.size();
    deliver(T.conns, out_conns, conn_capacity, nconn_out, "connections");
    deliver(T.bcs, out_bcs, bc_capacity, nbc_out, "boundary patches");
  });
}

cfd_status cfd_regroup(int32_t n, const int64_t* load, int32_t ngroups, const double* capacity,
                       int32_t* group, int64_t* group_load) {
  return cfd::host_guarded([&] {
    if (n < 0 || (n > 0 && (!load || !group))) host_fail(CFD_EINVAL, "bad load or group array");
    if (ngroups < 1) host_fail(CFD_EINVAL, "ngroups must be positive");
    for (int i = 0; i < n; ++i)
      if (load[i] < 0) host_fail(CFD_EINVAL, "load " + std::to_string(i) + " is negative");
    std::vector<double> cap(ngroups, 1.0);
    if (capacity)
      for (int g = 0; g < ngroups; ++g) {
        if (!(capacity[g] > 0.0) || !std::isfinite(capacity[g]))
          host_fail(CFD_EINVAL, "capacity " + std::to_string(g) + " must be positive and finite");
        cap[g] = capacity[g];
      }
    std::vector<int32_t> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return load[a] > load[b]; });
    std::vector<int64_t> total(ngroups, 0);
    for (int32_t i : order) {
      int best = 0;
      double best_v = (double)(total[0] + load[i]) / cap[0];
      for (int g = 1; g < ngroups; ++g) {
        const double v = (double)(total[g] + load[i]) / cap[g];
        if (v < best_v) best = g, best_v = v;
      }
      group[i] = best;
      total[best] += load[i];
    }
    if (group_load) std::copy(total.begin(), total.end(), group_load);
  });
}

}  // extern "C"
