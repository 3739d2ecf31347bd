// Host octree construction for the device hot path.
//
// Paper Sec. 4.2: the tree is refined top-down from the root by a predicate on
// each octant and then 2:1 balanced.  Paper Sec. 4.3: independent nodes are
// found from the leaf corners; a corner that coincides with a point one level
// below the corners of a coarser touching leaf (the paper's "cancellation
// nodes") is hanging and is re-expressed through that leaf's face or edge
// corners (Fig. 1 caption: hanging values come from the immediate parent).
//
// Single-process design: leaves live in an open-addressing hash set keyed by
// (level, Morton code); balancing walks the levels from finest to coarsest and
// splits any leaf that is more than one level coarser than the parent
// neighbourhood of a finer leaf, which yields the unique coarsest vertex-
// balanced refinement in one sweep.  Node de-duplication uses a radix sort of
// corner keys.  Leaves are then grouped into bricks (aligned cubes of 8^d,
// 4^d, 2^d leaves of one level, then single leaves) that the device kernels
// stream over without any per-leaf index map.
#include "mesh_host.h"

#include "brick_geom.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <thread>

namespace chns {
namespace {

inline uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}
inline uint64_t spread2(uint64_t x) {
  x &= 0xffffffffull;
  x = (x | x << 16) & 0x0000ffff0000ffffull;
  x = (x | x << 8) & 0x00ff00ff00ff00ffull;
  x = (x | x << 4) & 0x0f0f0f0f0f0f0f0full;
  x = (x | x << 2) & 0x3333333333333333ull;
  x = (x | x << 1) & 0x5555555555555555ull;
  return x;
}
inline uint64_t morton(int dim, const int32_t* c) {
  if (dim == 3) return spread3(c[0]) | spread3(c[1]) << 1 | spread3(c[2]) << 2;
  return spread2(c[0]) | spread2(c[1]) << 1;
}
inline uint64_t leaf_key(int dim, int level, const int32_t* a) {
  return ((uint64_t)level << 58) | morton(dim, a);
}
inline uint64_t mix(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Open-addressing hash set of 64-bit keys (erase by tombstone).
class KeySet {
 public:
  explicit KeySet(size_t expect) { rehash(std::max<size_t>(64, expect * 2)); }
  bool contains(uint64_t k) const {
    size_t i = mix(k) & mask_;
    while (true) {
      uint64_t v = slots_[i];
      if (v == kEmpty) return false;
      if (v == k) return true;
      i = (i + 1) & mask_;
    }
  }
  void insert(uint64_t k) {
    if ((used_ + 1) * 2 > slots_.size()) rehash(slots_.size() * 2);
    size_t i = mix(k) & mask_;
    size_t tomb = SIZE_MAX;
    while (true) {
      uint64_t v = slots_[i];
      if (v == k) return;
      if (v == kTomb && tomb == SIZE_MAX) tomb = i;
      if (v == kEmpty) break;
      i = (i + 1) & mask_;
    }
    if (tomb != SIZE_MAX) {
      slots_[tomb] = k;
    } else {
      slots_[i] = k;
      ++used_;
    }
  }
  void erase(uint64_t k) {
    size_t i = mix(k) & mask_;
    while (true) {
      uint64_t v = slots_[i];
      if (v == kEmpty) return;
      if (v == k) {
        slots_[i] = kTomb;
        return;
      }
      i = (i + 1) & mask_;
    }
  }
  // n keys inserted from several threads at once (insert_parallel below)
  template <typename F>
  void insert_parallel(int64_t n, F key_of);

 private:
  static constexpr uint64_t kEmpty = ~0ull;
  static constexpr uint64_t kTomb = ~0ull - 1;
  void rehash(size_t cap) {
    size_t c = 64;
    while (c < cap) c <<= 1;
    std::vector<uint64_t> old;
    old.swap(slots_);
    slots_.assign(c, kEmpty);
    mask_ = c - 1;
    used_ = 0;
    for (uint64_t v : old)
      if (v != kEmpty && v != kTomb) insert(v);
  }
  std::vector<uint64_t> slots_;
  size_t mask_ = 0;
  size_t used_ = 0;
};

bool box_meets_shell(const double* lo, const double* hi, const double* c, int dim, double r_in,
                     double r_out) {
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int d = 0; d < dim; ++d) {
    double nearest = std::min(std::max(c[d], lo[d]), hi[d]);
    dmin2 += (nearest - c[d]) * (nearest - c[d]);
    double far = std::max(std::fabs(lo[d] - c[d]), std::fabs(hi[d] - c[d]));
    dmax2 += far * far;
  }
  if (dmin2 > r_out * r_out) return false;
  if (r_in > 0.0 && dmax2 < r_in * r_in) return false;
  return true;
}

// Run f(t, begin, end) over T contiguous chunks of [0, n) on up to 16 host
// threads (fewer for small n); chunk t is always [n t / T, n (t + 1) / T),
// so work split this way and merged in chunk order is deterministic.  f must
// not throw.
template <typename F>
void parallel_chunks(int64_t n, int64_t min_per_thread, F f) {
  int64_t T = std::min<int64_t>(16, std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency()));
  T = std::max<int64_t>(1, std::min<int64_t>(T, n / std::max<int64_t>(1, min_per_thread)));
  std::vector<std::thread> th;
  int64_t started = 1;
  try {
    for (int64_t t = 1; t < T; ++t) {
      th.emplace_back([&f, t, T, n] { f(t, n * t / T, n * (t + 1) / T); });
      ++started;
    }
  } catch (...) {
    // fewer threads than asked for: the remaining chunks run here
  }
  for (int64_t t = started; t < T; ++t) f(t, n * t / T, n * (t + 1) / T);
  f(0, 0, n / T);
  for (auto& x : th) x.join();
}
inline int64_t chunk_count(int64_t n, int64_t min_per_thread) {
  int64_t T = std::min<int64_t>(16, std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency()));
  return std::max<int64_t>(1, std::min<int64_t>(T, n / std::max<int64_t>(1, min_per_thread)));
}

// Lock-free linear probing: a thread claims an empty slot by compare-and-swap
// and, when another key took it first, probes on.  The set's contents do not
// depend on the threads' order (only where a key sits in the table does),
// and the table is sized first, so no rehash runs meanwhile.
template <typename F>
void KeySet::insert_parallel(int64_t n, F key_of) {
  while ((used_ + (size_t)n + 1) * 2 > slots_.size()) rehash(slots_.size() * 2);
  uint64_t* sl = slots_.data();
  const size_t mask = mask_;
  std::vector<int64_t> added((size_t)chunk_count(n, 1 << 14), 0);
  parallel_chunks(n, 1 << 14, [&](int64_t t, int64_t a, int64_t b) {
    int64_t add = 0;
    for (int64_t e = a; e < b; ++e) {
      const uint64_t k = key_of(e);
      size_t i = mix(k) & mask;
      while (true) {
        const uint64_t v = __atomic_load_n(&sl[i], __ATOMIC_RELAXED);
        if (v == k) break;
        if (v == kEmpty) {
          uint64_t expect = kEmpty;
          if (__atomic_compare_exchange_n(&sl[i], &expect, k, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
            ++add;
            break;
          }
          if (expect == k) break;
        }
        i = (i + 1) & mask;
      }
    }
    added[(size_t)t] = add;
  });
  for (int64_t a : added) used_ += (size_t)a;
}

// Stable LSD radix sort of (key, val) pairs by the low key_bits of key:
// per-chunk digit histograms, then each chunk scatters its elements in order
// to offsets that put chunk t's elements of a digit after chunk t-1's.
void radix_sort_pairs(std::vector<uint64_t>& key, std::vector<uint32_t>& val, int key_bits) {
  const int64_t n = (int64_t)key.size();
  std::vector<uint64_t> k2((size_t)n);
  std::vector<uint32_t> v2((size_t)n);
  const int R = 11, NB = 1 << R;
  constexpr int64_t kMin = 1 << 16;
  const int64_t T = chunk_count(n, kMin);
  std::vector<int64_t> hist((size_t)(T * NB));
  for (int shift = 0; shift < key_bits; shift += R) {
    std::fill(hist.begin(), hist.end(), 0);
    parallel_chunks(n, kMin, [&](int64_t t, int64_t a, int64_t b) {
      int64_t* h = &hist[(size_t)(t * NB)];
      for (int64_t i = a; i < b; ++i) ++h[(key[(size_t)i] >> shift) & (NB - 1)];
    });
    // exclusive offsets in (digit, chunk) order
    int64_t run = 0;
    for (int d = 0; d < NB; ++d)
      for (int64_t t = 0; t < T; ++t) {
        const int64_t c = hist[(size_t)(t * NB + d)];
        hist[(size_t)(t * NB + d)] = run;
        run += c;
      }
    parallel_chunks(n, kMin, [&](int64_t t, int64_t a, int64_t b) {
      int64_t* h = &hist[(size_t)(t * NB)];
      for (int64_t i = a; i < b; ++i) {
        const int64_t p = h[(key[(size_t)i] >> shift) & (NB - 1)]++;
        k2[(size_t)p] = key[(size_t)i];
        v2[(size_t)p] = val[(size_t)i];
      }
    });
    key.swap(k2);
    val.swap(v2);
  }
}

struct Builder {
  const chns_mesh_spec& sp;
  HostMesh& m;
  std::string& msg;
  int dim, L;
  int32_t side;
  int nc;  // corners per leaf

  int32_t box_hi[3];  // domain box (units of 2^-L)
  bool carved;

  Builder(const chns_mesh_spec& s, HostMesh& mm, std::string& e)
      : sp(s), m(mm), msg(e), dim(s.dim), L(s.max_level), side(1 << s.max_level), nc(1 << s.dim) {
    carved = s.carve_level > 0;
    for (int d = 0; d < 3; ++d)
      box_hi[d] = (carved && d < dim && s.carve_level <= L) ? (s.extent[d] << (L - s.carve_level)) : side;
  }
  // octant (level lev, anchor a) lies outside the domain box
  bool outside(const int32_t* a) const {
    for (int d = 0; d < dim; ++d)
      if (a[d] >= box_hi[d]) return true;
    return false;
  }

  int32_t size_at(int lev) const { return side >> lev; }

  bool predicate(int lev, const int32_t* anc) {
    if (lev < sp.min_level) return true;
    if (lev >= L) return false;
    switch (sp.rule) {
      case CHNS_RULE_UNIFORM:
        return true;
      case CHNS_RULE_SPHERE_BAND:
      case CHNS_RULE_MULTI_SPHERE_BAND: {
        double lo[3], hi[3];
        for (int d = 0; d < dim; ++d) {
          lo[d] = (double)anc[d] / side;
          hi[d] = ((double)anc[d] + size_at(lev)) / side;
        }
        int ns = sp.rule == CHNS_RULE_SPHERE_BAND ? 1 : sp.n_spheres;
        for (int k = 0; k < ns; ++k) {
          double r = sp.radii[k];
          if (box_meets_shell(lo, hi, sp.centres + k * dim, dim, r - sp.band, r + sp.band)) return true;
        }
        return false;
      }
      case CHNS_RULE_CALLBACK: {
        int64_t a[3] = {anc[0], anc[1], dim == 3 ? anc[2] : 0};
        return sp.refine(a, lev, sp.user) != 0;
      }
    }
    return false;
  }

  // ---------------------------------------------------------------- refine
  void refine(std::vector<int8_t>& lev_out, std::vector<int32_t>& anc_out) {
    struct Item {
      int lev;
      int32_t a[3];
    };
    std::vector<Item> stack;
    stack.push_back({0, {0, 0, 0}});
    while (!stack.empty()) {
      Item it = stack.back();
      stack.pop_back();
      // carved octree: octants at or below the carve level lie wholly inside
      // or outside the box; the outside ones do not exist
      if (carved && it.lev >= sp.carve_level && outside(it.a)) continue;
      if (predicate(it.lev, it.a)) {
        int32_t h = size_at(it.lev + 1);
        // push children in reverse Morton order so that they pop in Morton order
        for (int c = nc - 1; c >= 0; --c) {
          Item ch{it.lev + 1, {0, 0, 0}};
          for (int d = 0; d < dim; ++d) ch.a[d] = it.a[d] + ((c >> d) & 1) * h;
          stack.push_back(ch);
        }
      } else {
        lev_out.push_back((int8_t)it.lev);
        for (int d = 0; d < 3; ++d) anc_out.push_back(it.a[d]);
      }
    }
  }

  // --------------------------------------------------------------- balance
  void balance(std::vector<int8_t>& lev, std::vector<int32_t>& anc) {
    const size_t n0 = lev.size();
    KeySet S(n0 * 2);
    S.insert_parallel((int64_t)n0, [&](int64_t i) { return leaf_key(dim, lev[i], &anc[3 * i]); });
    // the leaves of each level in leaf order: per-chunk counts, then each
    // chunk writes its leaves after the previous chunks'
    std::vector<std::vector<std::array<int32_t, 3>>> bylev(L + 1);
    {
      const int64_t T = chunk_count((int64_t)n0, 1 << 14);
      std::vector<std::vector<int64_t>> cnt((size_t)T, std::vector<int64_t>(L + 1, 0));
      parallel_chunks((int64_t)n0, 1 << 14, [&](int64_t t, int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) ++cnt[(size_t)t][lev[i]];
      });
      for (int l = 0; l <= L; ++l) {
        int64_t off = 0;
        for (int64_t t = 0; t < T; ++t) {
          const int64_t c = cnt[(size_t)t][l];
          cnt[(size_t)t][l] = off;
          off += c;
        }
        bylev[l].resize((size_t)off);
      }
      parallel_chunks((int64_t)n0, 1 << 14, [&](int64_t t, int64_t a, int64_t b) {
        std::vector<int64_t>& at = cnt[(size_t)t];
        for (int64_t i = a; i < b; ++i) bylev[lev[i]][(size_t)at[lev[i]]++] = {anc[3 * i], anc[3 * i + 1], anc[3 * i + 2]};
      });
    }
    auto align = [&](const int32_t* p, int l, int32_t* out) {
      int32_t s = size_at(l);
      for (int d = 0; d < 3; ++d) out[d] = d < dim ? (p[d] / s) * s : 0;
    };
    int ndir = 1;
    for (int d = 0; d < dim; ++d) ndir *= 3;
    // the leaf holding the point N (level < l-1 returned for a coarser leaf,
    // -1 when a leaf of level l-1 or finer holds it: no action)
    auto coarse_cover = [&](const int32_t* N, int l) -> int {
      int32_t am[3];
      for (int mlev = l - 1; mlev <= L; ++mlev) {
        align(N, mlev, am);
        if (S.contains(leaf_key(dim, mlev, am))) return -1;
      }
      for (int mlev = l - 2; mlev >= 0; --mlev) {
        align(N, mlev, am);
        if (S.contains(leaf_key(dim, mlev, am))) return mlev;
      }
      return -1;
    };
    struct Req {
      int32_t N[3];
    };
    for (int l = L; l >= 2; --l) {
      // the neighbour checks depend only on the parent block: the level-l
      // leaves' parents, each once (sorted by Morton key, first leaf kept)
      const int64_t nl = (int64_t)bylev[l].size();
      if (nl == 0) continue;
      std::vector<uint64_t> pk((size_t)nl);
      parallel_chunks(nl, 1 << 14, [&](int64_t, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
          const auto& a = bylev[l][(size_t)i];
          int32_t P[3];
          align(a.data(), l - 1, P);
          pk[(size_t)i] = S.contains(leaf_key(dim, l, a.data())) ? morton(dim, P) : ~0ull;
        }
      });
      std::vector<uint64_t> keys;
      std::vector<uint32_t> ids;
      for (int64_t i = 0; i < nl; ++i)
        if (pk[(size_t)i] != ~0ull) {
          keys.push_back(pk[(size_t)i]);
          ids.push_back((uint32_t)i);
        }
      radix_sort_pairs(keys, ids, dim * (L + 1));
      std::vector<uint32_t> par;
      for (size_t i = 0; i < keys.size(); ++i)
        if (i == 0 || keys[i] != keys[i - 1]) par.push_back(ids[i]);
      // read-only checks in parallel: the neighbour points of every parent
      // that a leaf coarser than l-1 holds, per chunk in parent order
      const int64_t np = (int64_t)par.size();
      const int64_t T = chunk_count(np, 1 << 12);
      std::vector<std::vector<Req>> req((size_t)T);
      const int32_t sP = size_at(l - 1);
      parallel_chunks(np, 1 << 12, [&](int64_t t, int64_t j0, int64_t j1) {
        for (int64_t j = j0; j < j1; ++j) {
          int32_t P[3];
          align(bylev[l][par[(size_t)j]].data(), l - 1, P);
          for (int tt0 = 0; tt0 < ndir; ++tt0) {
            int tt = tt0;
            bool zero = true, inside = true;
            Req r{{0, 0, 0}};
            for (int d = 0; d < dim; ++d) {
              const int dir = tt % 3 - 1;
              tt /= 3;
              if (dir) zero = false;
              r.N[d] = P[d] + dir * sP;
              if (r.N[d] < 0 || r.N[d] >= box_hi[d]) inside = false;
            }
            if (zero || !inside) continue;
            if (coarse_cover(r.N, l) >= 0) req[(size_t)t].push_back(r);
          }
        }
      });
      // splits in that order, each checked again against the leaves as split
      // so far: the leaf holding N is refined down to level l-1
      for (auto& rv : req)
        for (const Req& r : rv) {
          const int cover = coarse_cover(r.N, l);
          if (cover < 0) continue;
          int32_t am[3];
          for (int mlev = cover; mlev < l - 1; ++mlev) {
            align(r.N, mlev, am);
            S.erase(leaf_key(dim, mlev, am));
            int32_t h = size_at(mlev + 1);
            for (int c = 0; c < nc; ++c) {
              std::array<int32_t, 3> ch = {0, 0, 0};
              for (int d = 0; d < dim; ++d) ch[d] = am[d] + ((c >> d) & 1) * h;
              S.insert(leaf_key(dim, mlev + 1, ch.data()));
              bylev[mlev + 1].push_back(ch);
            }
          }
        }
    }
    // collect the leaves that remain (level by level, in list order) and sort
    // them by the Morton key of the anchor (= depth-first order)
    std::vector<int64_t> base(L + 2, 0);
    for (int l = 0; l <= L; ++l) base[l + 1] = base[l] + (int64_t)bylev[l].size();
    const int64_t NT = base[L + 1];
    std::vector<int64_t> pos((size_t)NT + 1, 0);
    for (int l = 0; l <= L; ++l)
      parallel_chunks((int64_t)bylev[l].size(), 1 << 14, [&](int64_t, int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i)
          pos[(size_t)(base[l] + i) + 1] = S.contains(leaf_key(dim, l, bylev[l][(size_t)i].data())) ? 1 : 0;
      });
    for (int64_t g = 0; g < NT; ++g) pos[(size_t)g + 1] += pos[(size_t)g];
    const int64_t NL = pos[(size_t)NT];
    std::vector<uint64_t> keys((size_t)NL);
    std::vector<uint32_t> ids((size_t)NL);
    std::vector<int8_t> lv((size_t)NL);
    std::vector<int32_t> an((size_t)NL * 3);
    for (int l = 0; l <= L; ++l)
      parallel_chunks((int64_t)bylev[l].size(), 1 << 14, [&](int64_t, int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
          const size_t g = (size_t)(base[l] + i);
          if (pos[g + 1] == pos[g]) continue;
          const size_t k = (size_t)pos[g];
          const auto& A = bylev[l][(size_t)i];
          keys[k] = morton(dim, A.data());
          ids[k] = (uint32_t)k;
          lv[k] = (int8_t)l;
          std::memcpy(&an[3 * k], A.data(), 3 * sizeof(int32_t));
        }
      });
    radix_sort_pairs(keys, ids, dim * (L + 1));
    // a leaf listed twice (same level and anchor) is kept once; the stable
    // sort leaves the copies next to each other
    std::vector<uint32_t> keep;
    keep.reserve((size_t)NL);
    for (int64_t i = 0; i < NL; ++i) {
      if (i > 0 && keys[(size_t)i] == keys[(size_t)i - 1] && lv[ids[(size_t)i]] == lv[ids[(size_t)i - 1]]) continue;
      keep.push_back(ids[(size_t)i]);
    }
    lev.resize(keep.size());
    anc.resize(keep.size() * 3);
    parallel_chunks((int64_t)keep.size(), 1 << 14, [&](int64_t, int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) {
        lev[(size_t)i] = lv[keep[(size_t)i]];
        std::memcpy(&anc[3 * (size_t)i], &an[3 * (size_t)keep[(size_t)i]], 3 * sizeof(int32_t));
      }
    });
  }

  uint64_t node_key(const int32_t* c) const {
    if (m.node_order == 1) return morton(dim, c);
    if (m.node_order == 2) {
      // aligned blocks of 8^d finest-grid points in Morton order, x fastest
      // inside a block
      int32_t b[3] = {0, 0, 0};
      uint64_t in = 0;
      for (int d = dim - 1; d >= 0; --d) {
        b[d] = c[d] >> 3;
        in = in * 8 + (uint64_t)(c[d] & 7);
      }
      return morton(dim, b) << (3 * dim) | in;
    }
    uint64_t s1 = (uint64_t)side + 1;
    uint64_t k = 0;
    for (int d = dim - 1; d >= 0; --d) k = k * s1 + (uint64_t)c[d];
    return k;
  }
  int node_key_bits() const {
    if (m.node_order == 1) return dim * (L + 1);
    if (m.node_order == 2) return dim * (L > 2 ? L + 1 : 3);
    double b = dim * std::log2((double)side + 1.0);
    return (int)std::ceil(b) + 1;
  }

  // ----------------------------------------------------------------- nodes
  int nodes(std::vector<int32_t>& elem_corner, std::vector<int32_t>& all_entry,
            std::vector<int32_t>& all_coords) {
    const int64_t E = m.n_elems();
    if ((uint64_t)E * nc >= (1ull << 32)) {
      msg = "mesh too large for 32-bit corner ids";
      return CHNS_EINVAL;
    }
    std::vector<uint64_t> key((size_t)E * nc);
    std::vector<uint32_t> pay((size_t)E * nc);
    parallel_chunks(E, 1 << 14, [&](int64_t, int64_t e0, int64_t e1) {
      for (int64_t e = e0; e < e1; ++e) {
        int32_t s = size_at(m.leaf_level[e]);
        for (int a = 0; a < nc; ++a) {
          int32_t c[3] = {0, 0, 0};
          for (int d = 0; d < dim; ++d) c[d] = m.leaf_anchor[3 * e + d] + ((a >> d) & 1) * s;
          key[e * nc + a] = node_key(c);
          pay[e * nc + a] = (uint32_t)(e * nc + a);
        }
      }
    });
    radix_sort_pairs(key, pay, node_key_bits());
    // distinct keys = nodes, numbered in key order: a run of equal keys is
    // one node (its coordinates from the run's first corner, its finest
    // touching level the largest over the run); runs are found per chunk and
    // numbered by prefix counts
    const int64_t NK = (int64_t)key.size();
    elem_corner.assign((size_t)NK, -1);
    const int64_t T = chunk_count(NK, 1 << 16);
    std::vector<int64_t> first((size_t)T + 1, 0);
    parallel_chunks(NK, 1 << 16, [&](int64_t t, int64_t a, int64_t b) {
      int64_t c = 0;
      for (int64_t i = a; i < b; ++i) c += (i == 0 || key[(size_t)i] != key[(size_t)i - 1]) ? 1 : 0;
      first[(size_t)t + 1] = c;
    });
    for (int64_t t = 0; t < T; ++t) first[(size_t)t + 1] += first[(size_t)t];
    const int64_t NA = first[(size_t)T];
    std::vector<uint64_t> ukey((size_t)NA);
    std::vector<int8_t> maxlev((size_t)NA);
    all_coords.assign((size_t)NA * 3, 0);
    parallel_chunks(NK, 1 << 16, [&](int64_t t, int64_t a, int64_t b) {
      int64_t id = first[(size_t)t] - 1;
      for (int64_t i = a; i < b; ++i) {
        if (i == 0 || key[(size_t)i] != key[(size_t)i - 1]) {
          ++id;
          ukey[(size_t)id] = key[(size_t)i];
          const uint32_t p = pay[(size_t)i];
          const int64_t e = p / nc;
          const int a2 = p % nc;
          const int32_t s = size_at(m.leaf_level[e]);
          for (int d = 0; d < dim; ++d)
            all_coords[3 * (size_t)id + d] = m.leaf_anchor[3 * e + d] + ((a2 >> d) & 1) * s;
          // the finest level over the run, which may continue past this chunk
          int8_t lm = m.leaf_level[e];
          for (int64_t j = i + 1; j < NK && key[(size_t)j] == key[(size_t)i]; ++j)
            lm = std::max(lm, m.leaf_level[pay[(size_t)j] / nc]);
          maxlev[(size_t)id] = lm;
        }
        elem_corner[pay[(size_t)i]] = (int32_t)id;
      }
    });
    key.clear();
    key.shrink_to_fit();
    pay.clear();
    pay.shrink_to_fit();

    // hanging detection: a corner that is not on the level-(lmax-1) grid and
    // that sits on the boundary of a level-(lmax-1) leaf is hanging.
    KeySet S((size_t)E * 2);
    S.insert_parallel(E, [&](int64_t e) { return leaf_key(dim, m.leaf_level[e], &m.leaf_anchor[3 * e]); });
    // the octant (corner direction o) of the coarse leaf holding each node,
    // found in parallel (read-only lookups), then numbered in node order
    auto coarse_anchor = [&](const int32_t* c, int o, int32_t S2, int32_t* a) {
      bool ok = true;
      for (int d = 0; d < 3; ++d) a[d] = 0;
      for (int d = 0; d < dim; ++d) {
        if ((o >> d) & 1) {
          if (c[d] >= box_hi[d]) ok = false;
          a[d] = (c[d] / S2) * S2;
        } else {
          if (c[d] <= 0) ok = false;
          a[d] = ((c[d] - 1) / S2) * S2;
        }
      }
      return ok;
    };
    std::vector<int8_t> hang_o(NA, -1);
    parallel_chunks(NA, 1 << 14, [&](int64_t, int64_t n0, int64_t n1) {
      for (int64_t n = n0; n < n1; ++n) {
        int lm = maxlev[n];
        if (lm < 1) continue;
        const int32_t* c = &all_coords[3 * n];
        int32_t S2 = size_at(lm - 1);
        bool odd = false;
        for (int d = 0; d < dim; ++d)
          if (c[d] % S2) odd = true;
        if (!odd) continue;
        for (int o = 0; o < nc; ++o) {
          int32_t a[3];
          if (!coarse_anchor(c, o, S2, a)) continue;
          if (S.contains(leaf_key(dim, lm - 1, a))) {
            hang_o[n] = (int8_t)o;
            break;
          }
        }
      }
    });
    // independent and hanging nodes numbered in key order (per-chunk counts)
    const int64_t TC = chunk_count(NA, 1 << 14);
    std::vector<int64_t> hc((size_t)TC + 1, 0);
    parallel_chunks(NA, 1 << 14, [&](int64_t t, int64_t a, int64_t b) {
      int64_t c = 0;
      for (int64_t n = a; n < b; ++n) c += hang_o[n] >= 0 ? 1 : 0;
      hc[(size_t)t + 1] = c;
    });
    for (int64_t t = 0; t < TC; ++t) hc[(size_t)t + 1] += hc[(size_t)t];
    const int64_t nh = hc[(size_t)TC], ni = NA - nh;
    all_entry.assign(NA, 0);
    m.indep_coords.assign((size_t)ni * 3, 0);
    parallel_chunks(NA, 1 << 14, [&](int64_t t, int64_t a, int64_t b) {
      int64_t h = hc[(size_t)t], i = a - hc[(size_t)t];
      for (int64_t n = a; n < b; ++n) {
        if (hang_o[n] >= 0) {
          all_entry[n] = -(int32_t)(++h);
        } else {
          all_entry[n] = (int32_t)i;
          for (int d = 0; d < 3; ++d) m.indep_coords[3 * (size_t)i + d] = all_coords[3 * n + d];
          ++i;
        }
      }
    });
    m.n_indep = ni;
    m.n_hanging = nh;
    m.hang_parents.assign(nh * 4, -1);
    m.hang_npar.assign(nh, 0);
    m.hang_coords.resize(nh * 3);
    // a hanging node's parents: the corners of the coarse leaf's face or edge
    // that holds it (read-only lookups, one hanging node per iteration)
    int err = 0;
    parallel_chunks(NA, 1 << 14, [&](int64_t, int64_t a0, int64_t a1) {
      for (int64_t n = a0; n < a1; ++n) {
        if (hang_o[n] < 0) continue;
        const int64_t h = -all_entry[n] - 1;
        const int32_t* c = &all_coords[3 * n];
        for (int d = 0; d < 3; ++d) m.hang_coords[3 * h + d] = c[d];
        const int32_t s = size_at(maxlev[n] - 1);
        int32_t A[3];
        coarse_anchor(c, hang_o[n], s, A);
        int nfree = 0;
        int fixedbit[3] = {0, 0, 0};
        bool isfree[3] = {false, false, false};
        for (int d = 0; d < dim; ++d) {
          const int32_t r = c[d] - A[d];
          if (r == 0) fixedbit[d] = 0;
          else if (r == s) fixedbit[d] = 1;
          else {
            isfree[d] = true;
            ++nfree;
          }
        }
        int np = 0;
        for (int comb = 0; comb < (1 << nfree); ++comb) {
          int32_t pc[3] = {0, 0, 0};
          int k = 0;
          for (int d = 0; d < dim; ++d) {
            const int bit = isfree[d] ? ((comb >> k++) & 1) : fixedbit[d];
            pc[d] = A[d] + bit * s;
          }
          const uint64_t pk = node_key(pc);
          const auto it = std::lower_bound(ukey.begin(), ukey.end(), pk);
          if (it == ukey.end() || *it != pk) {
            __atomic_fetch_or(&err, 1, __ATOMIC_RELAXED);
            break;
          }
          const int32_t pe = all_entry[it - ukey.begin()];
          if (pe < 0) {
            __atomic_fetch_or(&err, 2, __ATOMIC_RELAXED);
            break;
          }
          m.hang_parents[4 * h + np++] = pe;
        }
        m.hang_npar[h] = (int8_t)np;
      }
    });
    if (err & 1) {
      msg = "hanging-node parent is not a leaf corner";
      return CHNS_EINVAL;
    }
    if (err & 2) {
      msg = "hanging-node parent is itself hanging (tree not 2:1 balanced)";
      return CHNS_EINVAL;
    }
    return CHNS_OK;
  }

  // ---------------------------------------------------------------- bricks
  void bricks(const std::vector<int32_t>& elem_corner, const std::vector<int32_t>& all_entry,
              std::vector<std::vector<int32_t>>& brick_elems) {
    const int64_t E = m.n_elems();
    std::vector<uint8_t> taken(E, 0);
    // largest brick edge that still leaves >= 1024 bricks (enough wavefronts
    // to fill the GPU); a positive spec.brick_max overrides the choice
    int bmax = 1;
    for (int B = 8; B >= 1; B >>= 1) {
      int64_t per = 1;
      for (int d = 0; d < dim; ++d) per *= B;
      if (E / per >= 1024) {
        bmax = B;
        break;
      }
    }
    if (sp.brick_max > 0) bmax = sp.brick_max;
    for (int c = 0; c < kBrickClasses; ++c) {
      BrickClass& bc = m.cls[c];
      int B = brick_side(c);
      int b = 3 - c;
      bc.B = B;
      int n = 1, np = 1;
      for (int d = 0; d < dim; ++d) {
        n *= B;
        np *= (B + 1);
      }
      bc.nodes_per_brick = np;
      // boundary ranks in lexicographic order of brick-local positions
      bc.rank.assign(np, -1);
      int nb = 0;
      for (int p = 0; p < np; ++p) {
        int t = p;
        bool bnd = false;
        for (int d = 0; d < dim; ++d) {
          int pd = t % (B + 1);
          t /= (B + 1);
          if (pd == 0 || pd == B) bnd = true;
        }
        if (bnd) bc.rank[p] = nb++;
      }
      bc.bnd_per_brick = nb;
      // the kernels compute ranks arithmetically; they must match this table
      if (nb != brick_boundary_count(dim, B)) throw std::logic_error("brick boundary count");
      for (int p = 0; p < np; ++p) {
        if (bc.rank[p] < 0) continue;
        int jx = p % (B + 1), rest = p / (B + 1);
        int jy = dim == 3 ? rest % (B + 1) : 0, z = dim == 3 ? rest / (B + 1) : rest;
        if (brick_rank(dim, B, jx, jy, z) != bc.rank[p]) throw std::logic_error("brick rank formula");
      }
      std::vector<int32_t>& elist = brick_elems[c];
      // a leaf starts a brick of this class when it is free, aligned to the
      // brick edge, and the n leaves from it on are free, of its level and end
      // at the brick's far corner; same-level aligned blocks never overlap,
      // so the starts are found independently (per chunk, in leaf order) and
      // give what a scan that skips each found brick gives
      const int64_t T = chunk_count(E, 1 << 14);
      std::vector<std::vector<int32_t>> found((size_t)T);
      parallel_chunks(E, 1 << 14, [&](int64_t t, int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
          if (taken[i]) continue;
          if (c == kBrickClasses - 1) {
            found[(size_t)t].push_back((int32_t)i);
            continue;
          }
          const int l = m.leaf_level[i];
          const int32_t s = size_at(l);
          bool ok = B <= bmax && l >= b && i + n <= E;
          for (int d = 0; ok && d < dim; ++d)
            if (m.leaf_anchor[3 * i + d] % (B * s)) ok = false;
          for (int64_t j = i; ok && j < i + n; ++j)
            if (taken[j] || m.leaf_level[j] != l) ok = false;
          for (int d = 0; ok && d < dim; ++d)
            if (m.leaf_anchor[3 * (i + n - 1) + d] != m.leaf_anchor[3 * i + d] + (B - 1) * s) ok = false;
          if (ok) found[(size_t)t].push_back((int32_t)i);
        }
      });
      std::vector<int32_t> first;
      for (auto& f : found) first.insert(first.end(), f.begin(), f.end());
      bc.count = (int64_t)first.size();
      // each brick's leaves ordered by local lexicographic position
      elist.assign((size_t)bc.count * n, -1);
      parallel_chunks(bc.count, 1 << 10, [&](int64_t, int64_t k0, int64_t k1) {
        for (int64_t k = k0; k < k1; ++k) {
          const int64_t i = first[(size_t)k];
          const int32_t s = size_at(m.leaf_level[i]);
          for (int64_t j = i; j < i + n; ++j) {
            int lp = 0, mul = 1;
            for (int d = 0; d < dim; ++d) {
              lp += ((m.leaf_anchor[3 * j + d] - m.leaf_anchor[3 * i + d]) / s) * mul;
              mul *= B;
            }
            elist[(size_t)k * n + lp] = (int32_t)j;
            taken[j] = 1;
          }
        }
      });
      // tables
      bc.table.resize((size_t)bc.count * np);
      bc.level.resize(bc.count);
      bc.anchor.resize((size_t)bc.count * 3);
      parallel_chunks(bc.count, 1 << 10, [&](int64_t, int64_t k0, int64_t k1) {
      for (int64_t k = k0; k < k1; ++k) {
        const int32_t* els = &elist[(size_t)k * n];
        bc.level[k] = m.leaf_level[els[0]];
        for (int d = 0; d < 3; ++d) bc.anchor[3 * k + d] = m.leaf_anchor[3 * (size_t)els[0] + d];
        for (int p = 0; p < np; ++p) {
          int t = p, le = 0, mul = 1, a = 0;
          for (int d = 0; d < dim; ++d) {
            int pd = t % (B + 1);
            t /= (B + 1);
            int ed = pd < B ? pd : B - 1;
            le += ed * mul;
            mul *= B;
            a |= (pd - ed) << d;
          }
          bc.table[(size_t)k * np + p] = all_entry[elem_corner[(size_t)els[le] * nc + a]];
        }
      }
      });
      // finest-level 8^3 bricks whose nodes are numbered block by block
      // (every point of the blocks they touch is an independent node): node
      // numbers from eight block bases, checked against the table
      bc.abase.clear();
      if (dim == 3 && B == 8 && m.node_order == 2) {
        bc.abase.assign((size_t)bc.count * 8, -1);
        parallel_chunks(bc.count, 1 << 10, [&](int64_t, int64_t k0, int64_t k1) {
          for (int64_t k = k0; k < k1; ++k) {
            if (bc.level[k] != L) continue;
            const int32_t* t = &bc.table[(size_t)k * np];
            int32_t base[8];
            bool ok = true;
            for (int q = 0; q < 8 && ok; ++q) {
              base[q] = t[8 * (q & 1) + 9 * 8 * ((q >> 1) & 1) + 81 * 8 * ((q >> 2) & 1)];
              ok = base[q] >= 0;
            }
            for (int p = 0; p < np && ok; ++p) {
              const int jx = p % 9, jy = (p / 9) % 9, jz = p / 81;
              const int q = (jx >> 3) | ((jy >> 3) << 1) | ((jz >> 3) << 2);
              ok = t[p] == base[q] + (jx & 7) + 8 * (jy & 7) + 64 * (jz & 7);
            }
            if (ok)
              for (int q = 0; q < 8; ++q) bc.abase[(size_t)k * 8 + q] = base[q];
          }
        });
      }
    }
    int64_t base = 0;
    for (int c = 0; c < kBrickClasses; ++c) {
      m.cls[c].slot_base = base;
      base += m.cls[c].count * m.cls[c].bnd_per_brick;
    }
    m.n_slots = base;
  }

  int combine() {
    const int64_t N = m.n_indep;
    if (m.n_slots >= (1ll << 30)) {
      msg = "too many brick-boundary slots";
      return CHNS_EINVAL;
    }
    // every brick-boundary slot names the independent nodes it lands on (a
    // hanging node's parents, with its weight code in the top bits), in
    // (class, brick, position) order: per chunk of bricks, merged in chunk
    // order; interior nodes are counted (each must be interior to one brick)
    std::vector<int32_t> interior(N, 0);
    std::vector<uint64_t> key;
    std::vector<uint32_t> val;
    int bad = 0;
    for (int c = 0; c < kBrickClasses; ++c) {
      const BrickClass& bc = m.cls[c];
      // pushes per chunk of bricks (counted first, then written in place)
      auto pushes_of = [&](int64_t k, int p) -> int {
        const int32_t e = bc.table[(size_t)k * bc.nodes_per_brick + p];
        if (bc.rank[p] < 0) return 0;
        return e >= 0 ? 1 : m.hang_npar[-e - 1];
      };
      const int64_t T = chunk_count(bc.count, 1 << 10);
      std::vector<int64_t> off((size_t)T + 1, 0);
      parallel_chunks(bc.count, 1 << 10, [&](int64_t t, int64_t k0, int64_t k1) {
        int64_t cnt = 0;
        for (int64_t k = k0; k < k1; ++k)
          for (int p = 0; p < bc.nodes_per_brick; ++p) cnt += pushes_of(k, p);
        off[(size_t)t + 1] = cnt;
      });
      off[0] = (int64_t)key.size();
      for (int64_t t = 0; t < T; ++t) off[(size_t)t + 1] += off[(size_t)t];
      key.resize((size_t)off[(size_t)T]);
      val.resize((size_t)off[(size_t)T]);
      parallel_chunks(bc.count, 1 << 10, [&](int64_t t, int64_t k0, int64_t k1) {
        size_t w = (size_t)off[(size_t)t];
        for (int64_t k = k0; k < k1; ++k)
          for (int p = 0; p < bc.nodes_per_brick; ++p) {
            const int32_t e = bc.table[(size_t)k * bc.nodes_per_brick + p];
            const int r = bc.rank[p];
            if (r < 0) {
              if (e < 0) __atomic_store_n(&bad, 1, __ATOMIC_RELAXED);
              else __atomic_fetch_add(&interior[e], 1, __ATOMIC_RELAXED);
              continue;
            }
            const uint32_t slot = (uint32_t)(bc.slot_base + k * bc.bnd_per_brick + r);
            if (e >= 0) {
              key[w] = (uint64_t)e;
              val[w++] = slot;
            } else {
              const int64_t h = -e - 1;
              const int np = m.hang_npar[h];
              const uint32_t code = np == 2 ? 1u : (np == 4 ? 2u : 0u);
              for (int q = 0; q < np; ++q) {
                key[w] = (uint64_t)m.hang_parents[4 * h + q];
                val[w++] = slot | (code << 30);
              }
            }
          }
      });
    }
    if (bad) {
      msg = "hanging node inside a brick";
      return CHNS_EINVAL;
    }
    // grouped by node, each node's entries in that order (stable sort)
    int bits = 1;
    while (bits < 63 && (1ll << bits) <= N) ++bits;
    radix_sort_pairs(key, val, bits);
    const int64_t P = (int64_t)key.size();
    std::vector<int32_t> cnt(N + 1, 0);
    for (int64_t j = 0; j < P; ++j) ++cnt[(size_t)key[(size_t)j] + 1];
    for (int64_t i = 0; i < N; ++i) {
      bool in = interior[i] > 0, sh = cnt[i + 1] > 0;
      if (interior[i] > 1 || in == sh) {
        msg = "node ownership is inconsistent";
        return CHNS_EINVAL;
      }
    }
    m.comb_ent.assign(val.begin(), val.end());
    m.comb_ptr.push_back(0);
    for (int64_t i = 0; i < N; ++i) {
      if (cnt[i + 1] == 0) continue;
      m.comb_node.push_back((int32_t)i);
      m.comb_ptr.push_back(m.comb_ptr.back() + cnt[i + 1]);
    }
    return CHNS_OK;
  }

  // colouring such that no two nodes of one colour are coupled by any leaf
  int colour(const std::vector<int32_t>& elem_corner, const std::vector<int32_t>& all_entry) {
    const int64_t N = m.n_indep, E = m.n_elems();
    m.color.assign(N, 0);
    if (m.uniform) {
      int32_t s = size_at(L);
      for (int64_t i = 0; i < N; ++i) {
        int c = 0;
        for (int d = 0; d < dim; ++d) c |= ((m.indep_coords[3 * i + d] / s) & 1) << d;
        m.color[i] = (uint8_t)c;
      }
      m.n_colors = 1 << dim;
      return CHNS_OK;
    }
    auto expand = [&](int64_t e, int32_t* out) {
      int k = 0;
      for (int a = 0; a < nc; ++a) {
        int32_t v = all_entry[elem_corner[e * nc + a]];
        if (v >= 0) {
          out[k++] = v;
        } else {
          int64_t h = -v - 1;
          for (int q = 0; q < m.hang_npar[h]; ++q) out[k++] = m.hang_parents[4 * h + q];
        }
      }
      std::sort(out, out + k);
      return (int)(std::unique(out, out + k) - out);
    };
    // every leaf's coupled independent nodes (hanging corners replaced by
    // their parents), sorted and unique: lengths, then the lists, in parallel
    std::vector<int64_t> eptr(E + 1, 0);
    parallel_chunks(E, 1 << 14, [&](int64_t, int64_t e0, int64_t e1) {
      int32_t buf[64];
      for (int64_t e = e0; e < e1; ++e) eptr[e + 1] = expand(e, buf);
    });
    for (int64_t e = 0; e < E; ++e) eptr[e + 1] += eptr[e];
    std::vector<int32_t> eent((size_t)eptr[E]);
    parallel_chunks(E, 1 << 14, [&](int64_t, int64_t e0, int64_t e1) {
      // the raw list (before removing duplicates) may be longer than the
      // leaf's slot: expand into a buffer, copy the unique entries
      int32_t buf[64];
      for (int64_t e = e0; e < e1; ++e) {
        const int k = expand(e, buf);
        std::copy(buf, buf + k, &eent[(size_t)eptr[e]]);
      }
    });
    // the leaves around each node (counted and placed by atomic increments
    // from several threads: the order inside a node's list varies, the
    // colouring below only forms the union of their nodes' colours)
    std::vector<int32_t> cnt(N + 1, 0);
    parallel_chunks((int64_t)eent.size(), 1 << 16, [&](int64_t, int64_t a, int64_t b) {
      for (int64_t j = a; j < b; ++j) __atomic_fetch_add(&cnt[(size_t)eent[(size_t)j] + 1], 1, __ATOMIC_RELAXED);
    });
    for (int64_t i = 0; i < N; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> inc(cnt[N]);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    parallel_chunks(E, 1 << 14, [&](int64_t, int64_t e0, int64_t e1) {
      for (int64_t e = e0; e < e1; ++e)
        for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j)
          inc[(size_t)__atomic_fetch_add(&fill[(size_t)eent[(size_t)j]], 1, __ATOMIC_RELAXED)] = (int32_t)e;
    });
    // greedy colouring in node order
    std::vector<int16_t> col(N, -1);
    int maxc = 0;
    for (int64_t i = 0; i < N; ++i) {
      uint64_t used[4] = {0, 0, 0, 0};
      for (int32_t t = cnt[i]; t < cnt[i + 1]; ++t) {
        const int64_t e = inc[t];
        for (int64_t j = eptr[e]; j < eptr[e + 1]; ++j) {
          int16_t cj = col[eent[(size_t)j]];
          if (cj >= 0) used[cj >> 6] |= 1ull << (cj & 63);
        }
      }
      int c = 0;
      while (c < 256 && ((used[c >> 6] >> (c & 63)) & 1)) ++c;
      if (c >= 256) {
        msg = "node colouring needs more than 256 colours";
        return CHNS_EINVAL;
      }
      col[i] = (int16_t)c;
      maxc = std::max(maxc, c + 1);
    }
    for (int64_t i = 0; i < N; ++i) m.color[i] = (uint8_t)col[i];
    m.n_colors = maxc;
    return CHNS_OK;
  }

  int run() {
    if (dim != 2 && dim != 3) {
      msg = "dim must be 2 or 3";
      return CHNS_EINVAL;
    }
    if (L < 1 || L > 16 || sp.min_level < 0 || sp.min_level > L) {
      msg = "need 0 <= min_level <= max_level, 1 <= max_level <= 16";
      return CHNS_EINVAL;
    }
    if ((sp.rule == CHNS_RULE_SPHERE_BAND || sp.rule == CHNS_RULE_MULTI_SPHERE_BAND) &&
        (!sp.centres || !sp.radii || (sp.rule == CHNS_RULE_MULTI_SPHERE_BAND && sp.n_spheres < 1))) {
      msg = "band rules need centres and radii";
      return CHNS_EINVAL;
    }
    if (sp.rule == CHNS_RULE_CALLBACK && !sp.refine) {
      msg = "callback rule needs refine()";
      return CHNS_EINVAL;
    }
    if (sp.rule < 0 || sp.rule > 3) {
      msg = "unknown rule";
      return CHNS_EINVAL;
    }
    if (carved) {
      bool ok = sp.carve_level <= sp.min_level && sp.carve_level <= L && sp.carve_level <= 16;
      for (int d = 0; d < dim && ok; ++d) ok = sp.extent[d] >= 1 && sp.extent[d] <= (1 << sp.carve_level);
      if (!ok) {
        msg = "carved octree needs 1 <= carve_level <= min_level and 1 <= extent[d] <= 2^carve_level";
        return CHNS_EINVAL;
      }
    } else if (sp.carve_level < 0) {
      msg = "carve_level must not be negative";
      return CHNS_EINVAL;
    }
    m.dim = dim;
    m.max_level = L;
    refine(m.leaf_level, m.leaf_anchor);
    if (m.leaf_level.empty()) {
      msg = "no octant inside the domain";
      return CHNS_EINVAL;
    }
    return finish();
  }

  // From an explicit leaf list already stored in m (levels, anchors).
  int run_leaves() {
    if (dim != 2 && dim != 3) {
      msg = "dim must be 2 or 3";
      return CHNS_EINVAL;
    }
    m.dim = dim;
    m.max_level = L;
    return finish();
  }

  int finish() {
    balance(m.leaf_level, m.leaf_anchor);
    int lmin = 99, lmax = -1;
    for (auto l : m.leaf_level) {
      lmin = std::min<int>(lmin, l);
      lmax = std::max<int>(lmax, l);
    }
    // "uniform" means the whole cube at one level: the structured kernels,
    // the stencil multigrid levels and the network grid rely on it
    m.uniform = lmin == lmax && lmax == L && !carved;
    m.carve_level = carved ? sp.carve_level : 0;
    for (int d = 0; d < 3; ++d) m.box_hi[d] = d < dim ? box_hi[d] : 0;
    // uniform meshes: lexicographic (the structured kernels index nodes by
    // coordinates); otherwise blocked, so that a brick's node rows are
    // mostly contiguous and its gathers touch few cache lines
    m.node_order = m.uniform ? 0 : 2;
    std::vector<int32_t> elem_corner, all_entry, all_coords;
    int rc = nodes(elem_corner, all_entry, all_coords);
    if (rc) return rc;
    std::vector<std::vector<int32_t>> brick_elems(kBrickClasses);
    bricks(elem_corner, all_entry, brick_elems);
    rc = combine();
    if (rc) return rc;
    rc = colour(elem_corner, all_entry);
    if (rc) return rc;
    m.wall.assign(m.n_indep, 0);
    for (int64_t i = 0; i < m.n_indep; ++i)
      for (int d = 0; d < dim; ++d) {
        int32_t c = m.indep_coords[3 * i + d];
        if (c == 0 || c == box_hi[d]) m.wall[i] = 1;
      }
    return CHNS_OK;
  }
};

}  // namespace

int build_host_mesh_from_leaves(int dim, int max_level, const std::vector<int8_t>& level,
                                const std::vector<int32_t>& anchor, HostMesh& m, std::string& msg,
                                const HostMesh* like) {
  try {
    chns_mesh_spec sp{};
    sp.dim = dim;
    sp.min_level = 0;
    sp.max_level = max_level;
    sp.rule = CHNS_RULE_UNIFORM;
    if (like && like->carve_level > 0) {
      if (max_level < like->carve_level) {
        msg = "a level of a carved octree must not be coarser than its carve level";
        return CHNS_EINVAL;
      }
      sp.carve_level = like->carve_level;
      for (int d = 0; d < dim; ++d) sp.extent[d] = like->box_hi[d] >> (like->max_level - like->carve_level);
    }
    Builder b(sp, m, msg);
    m.leaf_level = level;
    m.leaf_anchor = anchor;
    return b.run_leaves();
  } catch (const std::bad_alloc&) {
    msg = "host allocation failed while building a coarse mesh";
    return CHNS_ENOMEM;
  } catch (const std::logic_error& e) {
    msg = std::string("internal consistency check failed: ") + e.what();
    return CHNS_EINVAL;
  }
}

void truncate_leaves(const HostMesh& f, int k, std::vector<int8_t>& lev, std::vector<int32_t>& anc) {
  const int sh = f.max_level - k;
  lev.clear();
  anc.clear();
  for (int64_t e = 0; e < f.n_elems(); ++e) {
    int l = f.leaf_level[e];
    int8_t nl = (int8_t)std::min(l, k);
    int32_t a[3];
    for (int d = 0; d < 3; ++d) {
      int32_t v = f.leaf_anchor[3 * e + d] >> sh;
      // anchor of the level-nl ancestor in units of 2^-k
      const int32_t s = 1 << (k - nl);
      a[d] = (v / s) * s;
    }
    const size_t n = lev.size();
    if (n > 0 && lev[n - 1] == nl && anc[3 * n - 3] == a[0] && anc[3 * n - 2] == a[1] && anc[3 * n - 1] == a[2])
      continue;  // descendants of one ancestor are contiguous in Morton order
    lev.push_back(nl);
    anc.insert(anc.end(), a, a + 3);
  }
}

namespace {
// node coordinate -> entry (independent id >= 0, hanging -(h+1))
struct NodeLookup {
  std::vector<uint64_t> key;
  std::vector<int32_t> val;
  uint64_t s1;
  int dim;
  explicit NodeLookup(const HostMesh& m) : s1((uint64_t)(1 << m.max_level) + 1), dim(m.dim) {
    // keys of every node (distinct coordinates, so distinct keys), sorted
    // with their entries on several threads
    const int64_t ni = m.n_indep, nt = m.n_indep + m.n_hanging;
    key.resize((size_t)nt);
    std::vector<uint32_t> ids((size_t)nt);
    parallel_chunks(nt, 1 << 14, [&](int64_t, int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) {
        key[(size_t)i] = enc(i < ni ? &m.indep_coords[3 * i] : &m.hang_coords[3 * (i - ni)]);
        ids[(size_t)i] = (uint32_t)i;
      }
    });
    int bits = 1;
    while (bits < 63 && (uint64_t)1 << bits <= enc_max()) ++bits;
    radix_sort_pairs(key, ids, bits);
    val.resize((size_t)nt);
    parallel_chunks(nt, 1 << 14, [&](int64_t, int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) {
        const int64_t j = ids[(size_t)i];
        val[(size_t)i] = j < ni ? (int32_t)j : -(int32_t)(j - ni + 1);
      }
    });
  }
  uint64_t enc_max() const {
    uint64_t k = 0;
    for (int d = 0; d < dim; ++d) k = k * s1 + (s1 - 1);
    return k;
  }
  uint64_t enc(const int32_t* c) const {
    uint64_t k = 0;
    for (int d = dim - 1; d >= 0; --d) k = k * s1 + (uint64_t)c[d];
    return k;
  }
  bool find(const int32_t* c, int32_t* out) const {
    uint64_t k = enc(c);
    auto it = std::lower_bound(key.begin(), key.end(), k);
    if (it == key.end() || *it != k) return false;
    *out = val[it - key.begin()];
    return true;
  }
};

// a node entry (independent id, or -(h + 1) for hanging node h) with weight
// w, hanging nodes expanded into their parents (equal shares)
void expand_entry(const HostMesh& m, int32_t entry, double w, std::vector<std::pair<int32_t, double>>& row) {
  if (entry >= 0) {
    row.push_back({entry, w});
    return;
  }
  const int64_t h = -entry - 1;
  const int np = m.hang_npar[h];
  for (int q = 0; q < np; ++q) row.push_back({m.hang_parents[4 * h + q], w / np});
}
// sort by (column, value), sum duplicates in that order, drop zeros
void merge_row(std::vector<std::pair<int32_t, double>>& row) {
  std::sort(row.begin(), row.end());
  size_t w = 0;
  for (size_t r = 0; r < row.size(); ++r) {
    if (w > 0 && row[w - 1].first == row[r].first) row[w - 1].second += row[r].second;
    else row[w++] = row[r];
  }
  row.resize(w);
  w = 0;
  for (size_t r = 0; r < row.size(); ++r)
    if (row[r].second != 0.0) row[w++] = row[r];
  row.resize(w);
}

// CSR matrix built row by row on several host threads: row(i, entries)
// appends the entries of row i (any order, duplicates allowed) and returns
// false with msg set on an error; rows are merged and concatenated in order.
template <typename RowFn>
int build_rows(int64_t nrows, RowFn row, std::vector<int32_t>& ptr, std::vector<int32_t>& col,
               std::vector<double>& val, std::string& msg) {
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(16, std::min<int64_t>(
                                                                    (int64_t)std::thread::hardware_concurrency(),
                                                                    nrows / 4096 + 1)));
  struct Part {
    std::vector<int32_t> len, col;
    std::vector<double> val;
    std::string err;
  };
  std::vector<Part> parts((size_t)nt);
  auto work = [&](int64_t t) {
    // no exception may leave a worker thread
    Part& p = parts[(size_t)t];
    try {
      const int64_t a = nrows * t / nt, b = nrows * (t + 1) / nt;
      std::vector<std::pair<int32_t, double>> e;
      p.len.reserve((size_t)(b - a));
      for (int64_t i = a; i < b; ++i) {
        e.clear();
        if (!row(i, e, p.err)) return;
        merge_row(e);
        p.len.push_back((int32_t)e.size());
        for (auto& x : e) {
          p.col.push_back(x.first);
          p.val.push_back(x.second);
        }
      }
    } catch (const std::bad_alloc&) {
      p.err = "host allocation failed while building a transfer";
    } catch (...) {
      p.err = "internal error while building a transfer";
    }
  };
  std::vector<std::thread> th;
  int64_t started = 1;
  try {
    for (int64_t t = 1; t < nt; ++t) {
      th.emplace_back(work, t);
      ++started;
    }
  } catch (...) {
    // fewer threads than asked for: the remaining parts run here
  }
  for (int64_t t = started; t < nt; ++t) work(t);
  work(0);
  for (auto& x : th) x.join();
  for (auto& p : parts)
    if (!p.err.empty()) {
      msg = p.err;
      return CHNS_EINVAL;
    }
  ptr.assign(1, 0);
  ptr.reserve((size_t)nrows + 1);
  col.clear();
  val.clear();
  for (auto& p : parts) {
    for (int32_t l : p.len) ptr.push_back(ptr.back() + l);
    col.insert(col.end(), p.col.begin(), p.col.end());
    val.insert(val.end(), p.val.begin(), p.val.end());
  }
  return CHNS_OK;
}

// transpose of a CSR matrix (rows x cols): entries of each transposed row in
// increasing original row order
void csr_transpose(int64_t cols, const std::vector<int32_t>& ptr, const std::vector<int32_t>& col,
                   const std::vector<double>& val, std::vector<int32_t>& tptr, std::vector<int32_t>& tcol,
                   std::vector<double>& tval) {
  const int64_t rows = (int64_t)ptr.size() - 1;
  tptr.assign((size_t)cols + 1, 0);
  for (int32_t c : col) ++tptr[(size_t)c + 1];
  for (int64_t c = 0; c < cols; ++c) tptr[(size_t)c + 1] += tptr[(size_t)c];
  std::vector<int32_t> cur(tptr.begin(), tptr.end() - 1);
  tcol.resize(col.size());
  tval.resize(val.size());
  for (int64_t i = 0; i < rows; ++i)
    for (int32_t k = ptr[(size_t)i]; k < ptr[(size_t)i + 1]; ++k) {
      const int32_t pos = cur[(size_t)col[(size_t)k]]++;
      tcol[(size_t)pos] = (int32_t)i;
      tval[(size_t)pos] = val[(size_t)k];
    }
}

}  // namespace

int build_transfer(const HostMesh& fine, const HostMesh& coarse, Transfer& t, std::string& msg) {
  const int dim = fine.dim;
  if (coarse.max_level != fine.max_level - 1 || coarse.dim != dim) {
    msg = "transfer needs meshes one level apart";
    return CHNS_EINVAL;
  }
  const int Lc = coarse.max_level;
  const int nc = 1 << dim;
  KeySet leaves((size_t)coarse.n_elems() * 2);
  leaves.insert_parallel(coarse.n_elems(),
                         [&](int64_t e) { return leaf_key(dim, coarse.leaf_level[e], &coarse.leaf_anchor[3 * e]); });
  NodeLookup cl(coarse), fl(fine);
  // prolongation rows: fine independent node <- coarse Q1 field at its position
  int rc = build_rows(
      fine.n_indep,
      [&](int64_t i, std::vector<std::pair<int32_t, double>>& row, std::string& err) {
        const int32_t* x = &fine.indep_coords[3 * i];
        int found = -1;
        int32_t af[3] = {0, 0, 0}, ac[3] = {0, 0, 0};
        int32_t sf = 0;
        for (int mlev = Lc; mlev >= 0 && found < 0; --mlev) {
          sf = 1 << (fine.max_level - mlev);  // coarse octant edge in fine units
          for (int d = 0; d < dim; ++d) {
            const int32_t q2 = 2 * x[d] + (x[d] < fine.box_hi[d] ? 1 : -1);  // doubled, nudged inside
            af[d] = (q2 / (2 * sf)) * sf;
            ac[d] = af[d] / 2;
          }
          if (leaves.contains(leaf_key(dim, mlev, ac))) found = mlev;
        }
        if (found < 0) {
          err = "fine node outside the coarse mesh";
          return false;
        }
        for (int a = 0; a < nc; ++a) {
          double w = 1.0;
          int32_t cc[3] = {0, 0, 0};
          for (int d = 0; d < dim; ++d) {
            const int bit = (a >> d) & 1;
            const double xi = (double)(x[d] - af[d]) / sf;
            w *= bit ? xi : 1.0 - xi;
            cc[d] = ac[d] + bit * (sf / 2);
          }
          if (w == 0.0) continue;
          int32_t ent;
          if (!cl.find(cc, &ent)) {
            err = "coarse leaf corner missing";
            return false;
          }
          expand_entry(coarse, ent, w, row);
        }
        return true;
      },
      t.P_ptr, t.P_col, t.P_val, msg);
  if (rc) return rc;
  // restriction = transpose (coarse rows, fine columns in increasing order)
  csr_transpose(coarse.n_indep, t.P_ptr, t.P_col, t.P_val, t.R_ptr, t.R_col, t.R_val);
  // injection of nodal fields: coarse node value = fine field at that point
  return build_rows(
      coarse.n_indep,
      [&](int64_t j, std::vector<std::pair<int32_t, double>>& row, std::string& err) {
        int32_t xf[3] = {0, 0, 0};
        for (int d = 0; d < dim; ++d) xf[d] = 2 * coarse.indep_coords[3 * j + d];
        int32_t ent;
        if (!fl.find(xf, &ent)) {
          err = "coarse node is not a fine node";
          return false;
        }
        expand_entry(fine, ent, 1.0, row);
        return true;
      },
      t.I_ptr, t.I_col, t.I_val, msg);
}

int build_host_mesh(const chns_mesh_spec& spec, HostMesh& m, std::string& msg) {
  try {
    Builder b(spec, m, msg);
    return b.run();
  } catch (const std::bad_alloc&) {
    msg = "host allocation failed while building the mesh";
    return CHNS_ENOMEM;
  } catch (const std::logic_error& e) {
    msg = std::string("internal consistency check failed: ") + e.what();
    return CHNS_EINVAL;
  }
}

// ------------------------------------------------------------ remeshing
namespace {

// Range of a nodal field over the nodes inside half-open aligned octants:
// the nodes sorted by Morton key (the box of an aligned octant is one key
// range), with per-block minima and maxima for the range queries.
struct BandQuery {
  static constexpr int64_t kBlk = 1024;
  int dim, L;
  double thr;
  std::vector<uint64_t> key;
  std::vector<double> v, bmin, bmax;

  BandQuery(const HostMesh& m, const double* phi, double t) : dim(m.dim), L(m.max_level), thr(t) {
    const int64_t ni = m.n_indep, nt = m.n_indep + m.n_hanging;
    std::vector<double> val((size_t)nt);
    std::vector<uint32_t> ids((size_t)nt);
    key.resize((size_t)nt);
    parallel_chunks(nt, 1 << 14, [&](int64_t, int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) {
        ids[(size_t)i] = (uint32_t)i;
        if (i < ni) {
          key[(size_t)i] = morton(dim, &m.indep_coords[3 * i]);
          val[(size_t)i] = phi[i];
        } else {
          // a hanging node's value: the mean of its parents (its constraint)
          const int64_t h = i - ni;
          const int np = m.hang_npar[h];
          double s = 0.0;
          for (int q = 0; q < np; ++q) s += phi[m.hang_parents[4 * h + q]];
          key[(size_t)i] = morton(dim, &m.hang_coords[3 * h]);
          val[(size_t)i] = s / np;
        }
      }
    });
    // node keys are distinct, so the order is that of the keys alone
    radix_sort_pairs(key, ids, dim * (L + 1));
    v.resize((size_t)nt);
    parallel_chunks(nt, 1 << 14, [&](int64_t, int64_t a, int64_t b) {
      for (int64_t i = a; i < b; ++i) v[(size_t)i] = val[ids[(size_t)i]];
    });
    const int64_t nb = ((int64_t)v.size() + kBlk - 1) / kBlk;
    bmin.assign((size_t)nb, INFINITY);
    bmax.assign((size_t)nb, -INFINITY);
    for (size_t i = 0; i < v.size(); ++i) {
      bmin[i / kBlk] = std::min(bmin[i / kBlk], v[i]);
      bmax[i / kBlk] = std::max(bmax[i / kBlk], v[i]);
    }
  }
  // do the values of the keys in [lo, hi) span a range meeting [-thr, thr]?
  bool meets(uint64_t lo, uint64_t hi) const {
    int64_t a = std::lower_bound(key.begin(), key.end(), lo) - key.begin();
    const int64_t b = std::lower_bound(key.begin(), key.end(), hi) - key.begin();
    if (a >= b) return false;
    double mn = INFINITY, mx = -INFINITY;
    while (a < b) {
      if (a % kBlk == 0 && a + kBlk <= b) {
        mn = std::min(mn, bmin[a / kBlk]);
        mx = std::max(mx, bmax[a / kBlk]);
        a += kBlk;
      } else {
        mn = std::min(mn, v[a]);
        mx = std::max(mx, v[a]);
        ++a;
      }
    }
    return mx >= -thr && mn <= thr;
  }
};

int band_refine(const int64_t anchor[3], int level, void* user) {
  const BandQuery& q = *static_cast<const BandQuery*>(user);
  const int32_t a[3] = {(int32_t)anchor[0], (int32_t)anchor[1], (int32_t)anchor[2]};
  const uint64_t lo = morton(q.dim, a);
  return q.meets(lo, lo + (1ull << (q.dim * (q.L - level)))) ? 1 : 0;
}

}  // namespace

int build_host_mesh_remesh(const HostMesh& old, const double* phi, int min_level, double thr, int brick_max,
                           HostMesh& out, std::string& msg) {
  if (!phi || min_level < 0 || min_level > old.max_level || !(thr >= 0.0)) {
    msg = "remesh needs the phase field, 0 <= min_level <= max_level and threshold >= 0";
    return CHNS_EINVAL;
  }
  try {
    BandQuery q(old, phi, thr);
    chns_mesh_spec sp{};
    sp.dim = old.dim;
    sp.min_level = min_level;
    sp.max_level = old.max_level;
    if (old.carve_level > 0) {
      if (min_level < old.carve_level) {
        msg = "remesh of a carved octree needs min_level >= its carve level";
        return CHNS_EINVAL;
      }
      sp.carve_level = old.carve_level;
      for (int d = 0; d < old.dim; ++d) sp.extent[d] = old.box_hi[d] >> (old.max_level - old.carve_level);
    }
    sp.rule = CHNS_RULE_CALLBACK;
    sp.refine = band_refine;
    sp.user = &q;
    sp.brick_max = brick_max;
    return build_host_mesh(sp, out, msg);
  } catch (const std::bad_alloc&) {
    msg = "host allocation failed while remeshing";
    return CHNS_ENOMEM;
  }
}

namespace {
// The Q1 field of src (hanging constraints included) at the point x (units of
// 2^-max_level, inside src's box): the trilinear weights of the corners of the
// leaf whose box holds x, nudged inside at the box's far faces.
bool field_at(const HostMesh& src, const KeySet& leaves, const NodeLookup& sl, const int32_t* x,
              std::vector<std::pair<int32_t, double>>& row, std::string& err) {
  const int dim = src.dim, L = src.max_level, nc = 1 << dim;
  int32_t af[3] = {0, 0, 0};
  int32_t sf = 0;
  int found = -1;
  for (int lev = L; lev >= 0 && found < 0; --lev) {
    sf = 1 << (L - lev);
    for (int d = 0; d < dim; ++d) {
      const int32_t q2 = 2 * x[d] + (x[d] < src.box_hi[d] ? 1 : -1);
      af[d] = (q2 / (2 * sf)) * sf;
    }
    if (leaves.contains(leaf_key(dim, lev, af))) found = lev;
  }
  if (found < 0) {
    err = "node outside the source mesh";
    return false;
  }
  for (int a = 0; a < nc; ++a) {
    double w = 1.0;
    int32_t cc[3] = {0, 0, 0};
    for (int d = 0; d < dim; ++d) {
      const int bit = (a >> d) & 1;
      const double xi = (double)(x[d] - af[d]) / sf;
      w *= bit ? xi : 1.0 - xi;
      cc[d] = af[d] + bit * sf;
    }
    if (w == 0.0) continue;
    int32_t ent;
    if (!sl.find(cc, &ent)) {
      err = "source leaf corner missing";
      return false;
    }
    expand_entry(src, ent, w, row);
  }
  return true;
}
}  // namespace

int build_interp(const HostMesh& src, const HostMesh& dst, std::vector<int32_t>& ptr, std::vector<int32_t>& col,
                 std::vector<double>& val, std::string& msg) {
  if (src.dim != dst.dim || src.max_level != dst.max_level) {
    msg = "transfer needs meshes of the same dimension and max_level";
    return CHNS_EINVAL;
  }
  try {
    KeySet leaves((size_t)src.n_elems() * 2);
    leaves.insert_parallel(src.n_elems(),
                           [&](int64_t e) { return leaf_key(src.dim, src.leaf_level[e], &src.leaf_anchor[3 * e]); });
    NodeLookup sl(src);
    return build_rows(
        dst.n_indep,
        [&](int64_t i, std::vector<std::pair<int32_t, double>>& row, std::string& err) {
          return field_at(src, leaves, sl, &dst.indep_coords[3 * i], row, err);
        },
        ptr, col, val, msg);
  } catch (const std::bad_alloc&) {
    msg = "host allocation failed while building the transfer";
    return CHNS_ENOMEM;
  }
}

int build_grid_transfer(const HostMesh& m, int g, GridTransfer& t, std::string& msg) {
  if (m.dim != 3 || m.carve_level != 0 || g < 1 || g > m.max_level) {
    msg = "grid transfers need a 3D octree on the whole cube whose max_level is at least the grid level";
    return CHNS_EINVAL;
  }
  try {
    const int L = m.max_level;
    const int32_t s = 1 << (L - g), G = (1 << g) + 1, cmax = (1 << g) - 1;
    t.level = g;
    // P: the grid's Q1 field at every mesh node (trilinear in the grid cell
    // that holds it; the last cell along an axis takes its far face)
    int rc = build_rows(
        m.n_indep,
        [&](int64_t i, std::vector<std::pair<int32_t, double>>& row, std::string&) {
          const int32_t* x = &m.indep_coords[3 * i];
          int32_t c[3];
          double xi[3];
          for (int d = 0; d < 3; ++d) {
            c[d] = std::min(x[d] / s, cmax);
            xi[d] = (double)(x[d] - c[d] * s) / s;
          }
          for (int a = 0; a < 8; ++a) {
            double w = 1.0;
            int64_t k = 0, mul = 1;
            for (int d = 0; d < 3; ++d) {
              const int bit = (a >> d) & 1;
              w *= bit ? xi[d] : 1.0 - xi[d];
              k += (c[d] + bit) * mul;
              mul *= G;
            }
            if (w != 0.0) row.push_back({(int32_t)k, w});
          }
          return true;
        },
        t.P_ptr, t.P_col, t.P_val, msg);
    if (rc) return rc;
    const int64_t ng = (int64_t)G * G * G;
    csr_transpose(ng, t.P_ptr, t.P_col, t.P_val, t.R_ptr, t.R_col, t.R_val);
    // Q: the mesh's Q1 field at every grid point
    KeySet leaves((size_t)m.n_elems() * 2);
    leaves.insert_parallel(m.n_elems(), [&](int64_t e) { return leaf_key(m.dim, m.leaf_level[e], &m.leaf_anchor[3 * e]); });
    NodeLookup sl(m);
    return build_rows(
        ng,
        [&](int64_t j, std::vector<std::pair<int32_t, double>>& row, std::string& err) {
          const int32_t x[3] = {(int32_t)(j % G) * s, (int32_t)((j / G) % G) * s, (int32_t)(j / ((int64_t)G * G)) * s};
          return field_at(m, leaves, sl, x, row, err);
        },
        t.Q_ptr, t.Q_col, t.Q_val, msg);
  } catch (const std::bad_alloc&) {
    msg = "host allocation failed while building the grid transfers";
    return CHNS_ENOMEM;
  }
}

}  // namespace chns
