// DoF numbering, gather maps, transfer categories (host side).
#include "dofs.hpp"
#include "geometry.hpp"

#include <algorithm>
#include <cmath>
#include <thread>

#include "common.hpp"
#include "fe1d.hpp"
#include "slots.hpp"

namespace mfmg {

namespace {

// Interleave the bits of three 21-bit coordinates (Morton / Z order).
uint64_t spread3(uint64_t x) {
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}
uint64_t morton(uint64_t x, uint64_t y, uint64_t z) { return spread3(x) | spread3(y) << 1 | spread3(z) << 2; }

// Open-addressing hash map uint64 -> int32 (keys < 2^63).
struct HashMap {
  std::vector<uint64_t> keys;
  std::vector<int32_t> vals;
  uint64_t mask = 0;
  explicit HashMap(size_t expected) {
    size_t cap = 16;
    while (cap < 2 * expected + 16) cap <<= 1;
    keys.assign(cap, 0);
    vals.assign(cap, -1);
    mask = cap - 1;
  }
  static uint64_t mix(uint64_t z) {
    z ^= z >> 33;
    z *= 0xff51afd7ed558ccdull;
    z ^= z >> 33;
    return z;
  }
  // returns existing value or inserts `v`; `inserted` tells which
  int32_t find_or_insert(uint64_t key, int32_t v, bool& inserted) {
    const uint64_t tagged = key | (1ull << 63);
    uint64_t h = mix(key) & mask;
    while (true) {
      if (keys[h] == tagged) { inserted = false; return vals[h]; }
      if (keys[h] == 0) { keys[h] = tagged; vals[h] = v; inserted = true; return v; }
      h = (h + 1) & mask;
    }
  }
};

// Exact position code of GLL node a of interval i on level l (see mfmg.h).
int64_t code1d(int l, int64_t i, int a, int k) {
  if (a == 0) return 2 * (i << (20 - l));
  if (a == k) return 2 * ((i + 1) << (20 - l));
  if (k % 2 == 0 && 2 * a == k) return 2 * ((2 * i + 1) << (19 - l));
  return 2 * ((((static_cast<int64_t>(l) << 25) + i) * 16) + a) + 1;
}

struct EntityRec {
  int level;
  int64_t i, j, k;
  int slot;
  int32_t first_dof;
  uint64_t key;
  uint8_t around;  // cells of the mesh's level inside the domain that contain the entity
};

}  // namespace

bool LevelDofs::slot_hanging(int64_t c, int s) const { return mfmg::slot_hanging(mask[c], s); }

double CoefDesc::value(double x, double y, double z) const {
  switch (kind) {
    case 0: return p[0] > 0 ? p[0] : 1.0;
    case 1: {
      const double dx = x - p[0], dy = y - p[1], dz = z - p[2];
      return dx * dx + dy * dy + dz * dz <= p[3] * p[3] ? p[4] : p[5];
    }
    case 2: {
      const int64_t s = static_cast<int64_t>(std::floor((x - p[3]) / p[2])) +
                        static_cast<int64_t>(std::floor((y - p[3]) / p[2])) +
                        static_cast<int64_t>(std::floor((z - p[3]) / p[2]));
      return (s % 2 == 0) ? p[0] : p[1];
    }
    default: throw Error(MFMG_ERR_INVALID_ARG, "unknown coefficient kind");
  }
}

namespace {
// cell value of the coefficient over the finest mesh (children summed in the
// order x fastest, then divided by 8)
double cell_coef(const CoefDesc& cd, const Octree& fine, int l, int64_t i, int64_t j, int64_t k) {
  if (fine.is_refined(l, i, j, k)) {
    double s = 0.0;
    for (int ch = 0; ch < 8; ++ch)
      s += cell_coef(cd, fine, l + 1, 2 * i + (ch & 1), 2 * j + ((ch >> 1) & 1), 2 * k + ((ch >> 2) & 1));
    return s / 8.0;
  }
  const double h = fine.h(l);
  return cd.value(fine.lo + (i + 0.5) * h, fine.lo + (j + 0.5) * h, fine.lo + (k + 0.5) * h);
}
}  // namespace

uint32_t coef_mask_bits(double c) {
  MFMG_REQUIRE(c >= 1e-30 && c <= 1e30, MFMG_ERR_INVALID_ARG, "the coefficient must lie in [1e-30, 1e30]");
  return coef_bits(c);
}

LevelDofs build_level_dofs(const Octree& tree, int k, bool dirichlet, bool want_codes, int only_level,
                           const CoefDesc* coef, const Octree* coef_fine) {
  MFMG_REQUIRE(k >= 1 && k <= 6, MFMG_ERR_UNSUPPORTED, "degree must be in [1, 6]");
  LevelDofs L;
  L.k = k;
  L.h0 = (tree.hi - tree.lo) / tree.n0;
  const int top = tree.n_levels();  // leaves live on levels 0..top
  MFMG_REQUIRE((static_cast<int64_t>(tree.n0) << top) < (1ll << 19), MFMG_ERR_UNSUPPORTED,
               "mesh too fine for 21-bit entity coordinates");

  // cells along the Morton curve of their lower corner on the finest lattice
  const bool ls_level = only_level >= 0;
  std::vector<Cell> cells = ls_level ? tree.cells_of_level(only_level) : tree.leaves();
  {
    std::vector<std::pair<uint64_t, int64_t>> order(cells.size());
    for (size_t c = 0; c < cells.size(); ++c) {
      const Cell& x = cells[c];
      int s = top - x.level;
      order[c] = {morton(x.i << s, x.j << s, x.k << s), static_cast<int64_t>(c)};
    }
    std::sort(order.begin(), order.end());
    std::vector<Cell> sorted(cells.size());
    for (size_t c = 0; c < cells.size(); ++c) sorted[c] = cells[order[c].second];
    cells.swap(sorted);
  }
  const int64_t nc = static_cast<int64_t>(cells.size());
  L.n_cells = nc;
  L.cells = cells;
  L.mask.assign(nc, 0);
  L.ent.assign(N_SLOTS * nc, -1);
  L.ent_id.assign(N_SLOTS * nc, -1);

  // hanging faces / edges on the parent's outer boundary
  for (int64_t c = 0; c < nc; ++c) {
    const Cell& x = cells[c];
    uint32_t m = static_cast<uint32_t>(x.level) << MASK_LEVEL_SHIFT;
    if (ls_level) {
      m |= static_cast<uint32_t>((x.i & 1) | (x.j & 1) << 1 | (x.k & 1) << 2);
    } else if (x.level > 0) {
      const int64_t p[3] = {x.i, x.j, x.k};
      int s[3], o[3];
      for (int d = 0; d < 3; ++d) {
        s[d] = static_cast<int>(p[d] & 1);
        o[d] = s[d] ? 1 : -1;
        m |= static_cast<uint32_t>(s[d]) << d;
      }
      auto missing = [&](int dx, int dy, int dz) {
        int64_t a = x.i + dx, b = x.j + dy, cc = x.k + dz;
        if (!tree.inside(x.level, a, b, cc) || tree.exists(x.level, a, b, cc)) return false;
        MFMG_REQUIRE(tree.exists(x.level - 1, a >> 1, b >> 1, cc >> 1), MFMG_ERR_INVALID_ARG,
                     "mesh is not one-irregular");
        return true;
      };
      for (int d = 0; d < 3; ++d) {
        int off[3] = {0, 0, 0};
        off[d] = o[d];
        if (missing(off[0], off[1], off[2])) m |= 1u << (MASK_FACE_SHIFT + d);
      }
      for (int d = 0; d < 3; ++d) {
        const int e = d == 0 ? 1 : 0, f = d == 2 ? 1 : 2;
        int a1[3] = {0, 0, 0}, a2[3] = {0, 0, 0}, a3[3] = {0, 0, 0};
        a1[e] = o[e];
        a2[f] = o[f];
        a3[e] = o[e];
        a3[f] = o[f];
        if (missing(a1[0], a1[1], a1[2]) || missing(a2[0], a2[1], a2[2]) || missing(a3[0], a3[1], a3[2]))
          m |= 1u << (MASK_EDGE_SHIFT + d);
      }
    }
    m |= coef_mask_bits(coef ? cell_coef(*coef, coef_fine ? *coef_fine : tree, x.level, x.i, x.j, x.k) : 1.0);
    L.mask[c] = m;
    if (mask_hanging(m)) ++L.n_hanging_cells;
  }

  // entities (ids only), first-touch order over the cells
  const int64_t dmax = static_cast<int64_t>(2 * tree.n0) << top;
  HashMap map(static_cast<size_t>(nc) * 8 + 64);
  std::vector<EntityRec> ents;
  ents.reserve(static_cast<size_t>(nc) * 8);
  for (int64_t c = 0; c < nc; ++c) {
    const Cell& x = cells[c];
    const uint32_t m = L.mask[c];
    for (int s = 0; s < 26; ++s) {
      Cell owner = x;
      if (mfmg::slot_hanging(m, s)) owner = {x.level - 1, x.i >> 1, x.j >> 1, x.k >> 1};
      const int sh = top - owner.level;
      int64_t D[3];
      const int64_t q[3] = {owner.i, owner.j, owner.k};
      bool boundary = false;
      int around = 1;
      for (int d = 0; d < 3; ++d) {
        const int sd = slot_side(s, d);
        D[d] = sd < 0 ? (2 * q[d] + 1) << sh : (2 * (q[d] + sd)) << sh;
        if (sd >= 0 && (D[d] == 0 || D[d] == dmax)) boundary = true;
        if (sd >= 0 && D[d] != 0 && D[d] != dmax) around *= 2;
      }
      if (dirichlet && boundary) continue;
      const uint64_t key = (static_cast<uint64_t>(D[0]) << 42) | (static_cast<uint64_t>(D[1]) << 21) |
                           static_cast<uint64_t>(D[2]);
      bool inserted;
      int32_t id = map.find_or_insert(key, static_cast<int32_t>(ents.size()), inserted);
      if (inserted)
        ents.push_back({owner.level, owner.i, owner.j, owner.k, s, -1, key, static_cast<uint8_t>(around)});
      L.ent_id[s * nc + c] = id;
    }
  }
  const int64_t n_bent = static_cast<int64_t>(ents.size());  // boundary-of-cell entities
  for (int64_t c = 0; c < nc; ++c) {
    L.ent_id[26 * nc + c] = static_cast<int32_t>(n_bent + c);
    const int sh = top - cells[c].level;
    const uint64_t key = (static_cast<uint64_t>((2 * cells[c].i + 1) << sh) << 42) |
                         (static_cast<uint64_t>((2 * cells[c].j + 1) << sh) << 21) |
                         static_cast<uint64_t>((2 * cells[c].k + 1) << sh);
    ents.push_back({cells[c].level, cells[c].i, cells[c].j, cells[c].k, 26, -1, key, 1});
  }
  const int64_t ne = static_cast<int64_t>(ents.size());
  L.n_entities = ne;
  MFMG_REQUIRE(ne < (1ll << 31), MFMG_ERR_UNSUPPORTED, "too many entities");
  auto esize = [&](int64_t id) { return slot_size(ents[id].slot, k); };

  // batches: consecutive cells while the touched DoFs fit the LDS budget.  A
  // block evaluates `quantum` cells at a time, so a full batch is cut back to
  // a multiple of that many cells (the cut-off cells start the next batch).
  const int mcap = batch_mcap(k);
  const int64_t quantum = BATCH_QUANTIZE ? BATCH_WAVES * cells_per_wave(k + 1) : 1;
  std::vector<int32_t> stamp(ne, -1);
  L.batch_cell_off.assign(1, 0);
  {
    int64_t local = 0, in_batch = 0, start = 0;
    int32_t b = 0;
    auto added = [&](int64_t c) {
      int64_t add = 0;
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = L.ent_id[s * nc + c];
        if (id >= 0 && stamp[id] != b) add += esize(id);
      }
      return add;
    };
    for (int64_t c = 0; c < nc; ++c) {
      int64_t add = added(c);
      if (in_batch > 0 && (local + add > mcap || in_batch >= batch_max_cells(k))) {
        const int64_t keep = in_batch > quantum ? in_batch / quantum * quantum : in_batch;
        c = start + keep;
        L.batch_cell_off.push_back(static_cast<int32_t>(c));
        ++b;
        start = c;
        local = 0;
        in_batch = 0;
        add = added(c);
      }
      MFMG_REQUIRE(add <= mcap, MFMG_ERR_UNSUPPORTED, "cell exceeds the batch capacity");
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = L.ent_id[s * nc + c];
        if (id >= 0 && stamp[id] != b) stamp[id] = b;
      }
      local += add;
      ++in_batch;
    }
    if (nc > 0) L.batch_cell_off.push_back(static_cast<int32_t>(nc));
  }
  const int64_t nb = static_cast<int64_t>(L.batch_cell_off.size()) - 1;
  L.n_batches = nb;

  // within each batch, cells with hanging nodes first: the operator evaluates
  // several cells per wavefront, and a wavefront takes the hanging-node path
  // if any of its cells needs it
  {
    std::vector<int64_t> order(nc);
    for (int64_t b = 0; b < nb; ++b) {
      int64_t w = L.batch_cell_off[b];
      for (int pass = 0; pass < 2; ++pass)
        for (int64_t c = L.batch_cell_off[b]; c < L.batch_cell_off[b + 1]; ++c)
          if (mask_hanging(L.mask[c]) == (pass == 0)) order[w++] = c;
    }
    std::vector<Cell> cells2(nc);
    std::vector<uint32_t> mask2(nc);
    std::vector<int32_t> ent2(L.ent_id.size());
    for (int64_t c = 0; c < nc; ++c) {
      cells2[c] = L.cells[order[c]];
      mask2[c] = L.mask[order[c]];
      for (int s = 0; s < N_SLOTS; ++s) ent2[s * nc + c] = L.ent_id[s * nc + order[c]];
    }
    L.cells.swap(cells2);
    L.mask.swap(mask2);
    L.ent_id.swap(ent2);
  }

  // shared (touched by >= 2 batches) or exclusive
  std::vector<int32_t> n_touch(ne, 0);
  std::fill(stamp.begin(), stamp.end(), -1);
  for (int64_t b = 0; b < nb; ++b)
    for (int64_t c = L.batch_cell_off[b]; c < L.batch_cell_off[b + 1]; ++c)
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = L.ent_id[s * nc + c];
        if (id < 0 || stamp[id] == static_cast<int32_t>(b)) continue;
        stamp[id] = static_cast<int32_t>(b);
        ++n_touch[id];
      }

  // numbering: shared entities first (first touch), then exclusive per batch
  std::vector<int64_t> start(ne, -1);
  int64_t next = 0;
  for (int64_t c = 0; c < nc; ++c)
    for (int s = 0; s < N_SLOTS; ++s) {
      const int32_t id = L.ent_id[s * nc + c];
      if (id < 0 || n_touch[id] < 2 || start[id] >= 0) continue;
      start[id] = next;
      next += esize(id);
    }
  L.n_shared = next;
  L.batch_ex_off.assign(nb + 1, 0);
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t ex0 = next;
    for (int64_t c = L.batch_cell_off[b]; c < L.batch_cell_off[b + 1]; ++c)
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = L.ent_id[s * nc + c];
        if (id < 0 || n_touch[id] != 1 || start[id] >= 0) continue;
        start[id] = next;
        next += esize(id);
      }
    L.batch_ex_off[b + 1] = static_cast<int32_t>(L.batch_ex_off[b] + (next - ex0));
  }
  MFMG_REQUIRE(next < (1ll << 31), MFMG_ERR_UNSUPPORTED, "more than 2^31 DoFs on a level");
  L.n_dofs = next;
  for (int64_t c = 0; c < nc; ++c)
    for (int s = 0; s < N_SLOTS; ++s) {
      const int32_t id = L.ent_id[s * nc + c];
      L.ent[s * nc + c] = id < 0 ? -1 : static_cast<int32_t>(start[id]);
    }

  // batch-local layout: shared entities in global order (so that every
  // batch's partial sums, and with them the reduction's reads, follow the
  // global order of the shared DoFs), then the exclusive range in global order
  L.loc.assign(static_cast<size_t>(N_SLOTS) * nc, static_cast<uint16_t>(batch_mcap(k)));  // absent: zero block
  L.batch_sh_off.assign(nb + 1, 0);
  std::vector<int32_t> lstart(ne, -1);
  std::fill(stamp.begin(), stamp.end(), -1);
  std::vector<int32_t> bshared;
  for (int64_t b = 0; b < nb; ++b) {
    bshared.clear();
    for (int64_t c = L.batch_cell_off[b]; c < L.batch_cell_off[b + 1]; ++c)
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = L.ent_id[s * nc + c];
        if (id < 0 || n_touch[id] < 2 || stamp[id] == static_cast<int32_t>(b)) continue;
        stamp[id] = static_cast<int32_t>(b);
        bshared.push_back(id);
      }
    std::sort(bshared.begin(), bshared.end(), [&](int32_t a, int32_t c) { return start[a] < start[c]; });
    int64_t nsh = 0;
    for (int32_t id : bshared) {
      lstart[id] = static_cast<int32_t>(nsh);
      for (int t = 0; t < esize(id); ++t) L.sh_idx.push_back(static_cast<int32_t>(start[id] + t));
      nsh += esize(id);
    }
    L.batch_sh_off[b + 1] = static_cast<int32_t>(L.batch_sh_off[b] + nsh);
    const int64_t ex_global = L.n_shared + L.batch_ex_off[b];
    for (int64_t c = L.batch_cell_off[b]; c < L.batch_cell_off[b + 1]; ++c)
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = L.ent_id[s * nc + c];
        if (id < 0) continue;
        const int64_t ls = n_touch[id] >= 2 ? lstart[id] : nsh + (start[id] - ex_global);
        MFMG_REQUIRE(ls >= 0 && ls + esize(id) <= batch_mcap(k), MFMG_ERR_INVALID_ARG, "batch layout");
        L.loc[s * nc + c] = static_cast<uint16_t>(ls);
      }
  }
  // partial sums of shared DoF s at red_off[s] .. red_off[s+1]-1, in batch order
  L.red_off.assign(L.n_shared + 1, 0);
  for (int32_t g : L.sh_idx) ++L.red_off[g + 1];
  for (int64_t i = 0; i < L.n_shared; ++i) L.red_off[i + 1] += L.red_off[i];
  // partial sums are stored batch by batch (position p = batch-local shared
  // entry); red_idx lists, for each shared DoF in CSR order, its positions
  L.red_idx.assign(L.sh_idx.size(), 0);
  {
    std::vector<int32_t> fill(L.red_off.begin(), L.red_off.end() - 1);
    for (size_t p = 0; p < L.sh_idx.size(); ++p) L.red_idx[fill[L.sh_idx[p]]++] = static_cast<int32_t>(p);
  }
  for (size_t e = 0; e < ents.size(); ++e) ents[e].first_dof = static_cast<int32_t>(start[e]);
  L.ent_key.resize(ne);
  L.ent_first.resize(ne);
  L.ent_size.resize(ne);
  for (int64_t e = 0; e < ne; ++e) {
    L.ent_key[e] = ents[e].key;
    L.ent_first[e] = ents[e].first_dof;
    L.ent_size[e] = static_cast<int32_t>(esize(e));
  }
  if (ls_level) {
    // refinement edge: fewer cells of this level contain the entity than lie
    // around it inside the domain (the rest of its surroundings is covered by
    // coarser leaves)
    std::vector<uint8_t> count(ne, 0);
    L.ent_on_leaf.assign(ne, 0);
    for (int64_t c = 0; c < nc; ++c) {
      const Cell& x = L.cells[c];
      const bool leaf = !tree.is_refined(x.level, x.i, x.j, x.k);
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = L.ent_id[s * nc + c];
        if (id < 0) continue;
        if (s < 26) ++count[id];
        if (leaf) L.ent_on_leaf[id] = 1;
      }
    }
    L.ent_edge.assign(ne, 0);
    L.dof_edge.assign(L.n_dofs, 0);
    for (int64_t e = 0; e < ne; ++e) {
      if (ents[e].slot == 26 || count[e] >= ents[e].around) continue;
      L.ent_edge[e] = 1;
      for (int t = 0; t < L.ent_size[e]; ++t) L.dof_edge[L.ent_first[e] + t] = 1;
      L.n_edge_dofs += L.ent_size[e];
    }
  }

  if (!want_codes) return L;
  // exact node codes of every DoF
  L.codes.assign(3 * L.n_dofs, 0);
  auto emit = [&](int lv, int64_t ci, int64_t cj, int64_t ck, int s, int64_t first) {
    int64_t dof = first;
    const int sa = slot_side(s, 0), sb = slot_side(s, 1), sc = slot_side(s, 2);
    for (int c = (sc < 0 ? 1 : sc * k); c <= (sc < 0 ? k - 1 : sc * k); ++c)
      for (int b = (sb < 0 ? 1 : sb * k); b <= (sb < 0 ? k - 1 : sb * k); ++b)
        for (int a = (sa < 0 ? 1 : sa * k); a <= (sa < 0 ? k - 1 : sa * k); ++a) {
          L.codes[3 * dof + 0] = code1d(lv, ci, a, k);
          L.codes[3 * dof + 1] = code1d(lv, cj, b, k);
          L.codes[3 * dof + 2] = code1d(lv, ck, c, k);
          ++dof;
        }
  };
  for (const EntityRec& e : ents)
    if (e.first_dof >= 0) emit(e.level, e.i, e.j, e.k, e.slot, e.first_dof);
  return L;
}

namespace {
// Greedy colouring of n items, each touching the entities that ents_of lists
// (slot 26, the cell interior, is never shared and not listed): an item takes
// the lowest colour none of its entities has seen.  Returns the items in
// colour order (stable) and the colour ranges.
template <typename EntsOf>
void greedy_colours(int64_t n, int64_t n_entities, EntsOf ents_of, std::vector<int64_t>& order,
                    std::vector<int64_t>& off) {
  std::vector<uint64_t> used(static_cast<size_t>(n_entities), 0);
  std::vector<int8_t> colour(static_cast<size_t>(n));
  int32_t ids[26];
  int n_colours = 0;
  for (int64_t q = 0; q < n; ++q) {
    const int m = ents_of(q, ids);
    uint64_t forbidden = 0;
    for (int i = 0; i < m; ++i) forbidden |= used[ids[i]];
    MFMG_REQUIRE(forbidden != ~uint64_t(0), MFMG_ERR_UNSUPPORTED, "deterministic mode: more than 64 colours");
    const int c = __builtin_ctzll(~forbidden);
    for (int i = 0; i < m; ++i) used[ids[i]] |= uint64_t(1) << c;
    colour[q] = static_cast<int8_t>(c);
    n_colours = std::max(n_colours, c + 1);
  }
  off.assign(n_colours + 1, 0);
  for (int64_t q = 0; q < n; ++q) ++off[colour[q] + 1];
  for (int c = 0; c < n_colours; ++c) off[c + 1] += off[c];
  std::vector<int64_t> pos(off.begin(), off.end() - 1);
  order.assign(n, 0);
  for (int64_t q = 0; q < n; ++q) order[pos[colour[q]]++] = q;
}

// the entities (slots 0..25, Dirichlet left out) of cell c of level L
int cell_entities(const LevelDofs& L, int64_t c, int32_t* ids) {
  int m = 0;
  for (int s = 0; s < 26; ++s) {
    const int32_t id = L.ent_id[s * L.n_cells + c];
    if (id >= 0) ids[m++] = id;
  }
  return m;
}
}  // namespace

void colour_cells(const LevelDofs& L, std::vector<int32_t>& cells, std::vector<int64_t>& off) {
  std::vector<int64_t> order;
  greedy_colours(L.n_cells, L.n_entities, [&](int64_t c, int32_t* ids) { return cell_entities(L, c, ids); }, order,
                 off);
  cells.assign(order.begin(), order.end());
}

TransferDofs build_transfer(const LevelDofs& fine, const LevelDofs& coarse, bool polynomial, bool skip_unrefined,
                            bool coloured) {
  TransferDofs T;
  T.polynomial = polynomial;
  const int64_t nf = fine.n_cells, ncc = coarse.n_cells;
  // groups of fine cells, one per coarse cell
  std::vector<int64_t> group_start(ncc + 1, 0);
  std::vector<int32_t> group_cells;
  group_cells.reserve(nf);
  // lookup of fine cells by (level, key): the two levels order their cells
  // independently (by batches), also on equal meshes
  std::vector<std::pair<uint64_t, int32_t>> idx(nf);
  for (int64_t c = 0; c < nf; ++c) {
    const Cell& x = fine.cells[c];
    idx[c] = {(static_cast<uint64_t>(x.level) << 59) ^ cell_key(x.i, x.j, x.k), static_cast<int32_t>(c)};
  }
  std::sort(idx.begin(), idx.end());
  auto find = [&](int l, int64_t i, int64_t j, int64_t k) -> int32_t {
    uint64_t key = (static_cast<uint64_t>(l) << 59) ^ cell_key(i, j, k);
    auto it = std::lower_bound(idx.begin(), idx.end(), std::make_pair(key, static_cast<int32_t>(-1)));
    if (it != idx.end() && it->first == key) return it->second;
    return -1;
  };
  if (polynomial) {
    MFMG_REQUIRE(nf == ncc, MFMG_ERR_INVALID_ARG, "polynomial transfer needs equal meshes");
    for (int64_t c = 0; c < ncc; ++c) {
      const Cell& x = coarse.cells[c];
      const int32_t f = find(x.level, x.i, x.j, x.k);
      MFMG_REQUIRE(f >= 0, MFMG_ERR_INVALID_ARG, "polynomial transfer needs equal meshes");
      T.ident_coarse.push_back(static_cast<int32_t>(c));
      T.ident_fine.push_back(f);
      group_cells.push_back(f);
      group_start[c + 1] = group_start[c] + 1;
    }
  } else {
    for (int64_t c = 0; c < ncc; ++c) {
      const Cell& x = coarse.cells[c];
      int32_t f = find(x.level, x.i, x.j, x.k);
      if (f >= 0) {
        T.ident_coarse.push_back(static_cast<int32_t>(c));
        T.ident_fine.push_back(f);
        group_cells.push_back(f);
      } else if (skip_unrefined && find(x.level + 1, 2 * x.i, 2 * x.j, 2 * x.k) < 0) {
        // an active coarse cell of a local-smoothing level: no transfer group
      } else {
        T.refined_coarse.push_back(static_cast<int32_t>(c));
        for (int ch = 0; ch < 8; ++ch) {
          int32_t g = find(x.level + 1, 2 * x.i + (ch & 1), 2 * x.j + ((ch >> 1) & 1), 2 * x.k + ((ch >> 2) & 1));
          MFMG_REQUIRE(g >= 0, MFMG_ERR_INVALID_ARG, "fine mesh is not a refinement of the coarse mesh");
          group_cells.push_back(g);
        }
      }
      group_start[c + 1] = static_cast<int64_t>(group_cells.size());
    }
    const int64_t nr = static_cast<int64_t>(T.refined_coarse.size());
    T.refined_fine.assign(8 * nr, -1);
    int64_t r = 0;
    for (int64_t c = 0; c < ncc; ++c)
      if (group_start[c + 1] - group_start[c] == 8) {
        for (int ch = 0; ch < 8; ++ch) T.refined_fine[ch * nr + r] = group_cells[group_start[c] + ch];
        ++r;
      }
  }
  MFMG_REQUIRE(static_cast<int64_t>(group_cells.size()) == nf, MFMG_ERR_INVALID_ARG,
               "transfer groups do not cover the fine mesh");

  // valence: number of groups in which an entity appears unconstrained
  std::vector<uint8_t> count(fine.n_entities, 0);
  std::vector<int32_t> seen;
  for (int64_t g = 0; g < ncc; ++g) {
    seen.clear();
    for (int64_t q = group_start[g]; q < group_start[g + 1]; ++q) {
      const int32_t c = group_cells[q];
      for (int s = 0; s < N_SLOTS; ++s) {
        const int32_t id = fine.ent_id[s * nf + c];
        if (id < 0 || fine.slot_hanging(c, s)) continue;
        seen.push_back(id);
      }
    }
    std::sort(seen.begin(), seen.end());
    seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
    for (int32_t id : seen) {
      MFMG_REQUIRE(count[id] < TRANSFER_OWNER - 1, MFMG_ERR_INVALID_ARG, "valence overflow");
      ++count[id];
    }
  }
  T.valence.assign(N_SLOTS * nf, 0);
  for (int64_t c = 0; c < nf; ++c)
    for (int s = 0; s < N_SLOTS; ++s) {
      const int32_t id = fine.ent_id[s * nf + c];
      if (id < 0 || fine.slot_hanging(c, s)) continue;
      MFMG_REQUIRE(count[id] > 0 && count[id] < TRANSFER_OWNER, MFMG_ERR_INVALID_ARG,
                   "entity without a transfer group, or valence overflow");
      T.valence[s * nf + c] = count[id];
    }
  if (coloured) {  // group lists in colour order (the restriction's coarse entities)
    std::vector<int64_t> order;
    const std::vector<int32_t> ic = T.ident_coarse, jf = T.ident_fine;
    greedy_colours(static_cast<int64_t>(ic.size()), coarse.n_entities,
                   [&](int64_t q, int32_t* ids) { return cell_entities(coarse, ic[q], ids); }, order, T.ident_off);
    for (size_t q = 0; q < order.size(); ++q) {
      T.ident_coarse[q] = ic[order[q]];
      T.ident_fine[q] = jf[order[q]];
    }
    const int64_t nrg = static_cast<int64_t>(T.refined_coarse.size());
    const std::vector<int32_t> rc = T.refined_coarse, rf = T.refined_fine;
    greedy_colours(nrg, coarse.n_entities, [&](int64_t q, int32_t* ids) { return cell_entities(coarse, rc[q], ids); },
                   order, T.refined_off);
    for (int64_t q = 0; q < nrg; ++q) {
      T.refined_coarse[q] = rc[order[q]];
      for (int ch = 0; ch < 8; ++ch) T.refined_fine[ch * nrg + q] = rf[ch * nrg + order[q]];
    }
  }
  // owner: of the (fine cell, slot) pairs through which the transfer kernels
  // reach an unconstrained entity, the first one (identity groups, then
  // refinement groups, nodes in lattice order); every other pair skips it.
  // A refinement group's lattice has 2k+1 nodes per axis, node I belonging
  // to child I >= k (local node I - k), so an entity on a face between
  // children is reached through one child only.
  const int kf = fine.k;
  std::vector<uint8_t> claimed(fine.n_entities, 0);
  auto visit = [&](int64_t f, int a, int b, int c) {
    const int s = node_slot(a, b, c, kf);
    uint8_t& v = T.valence[s * nf + f];
    if (v == 0) return;  // constrained or Dirichlet
    const int32_t id = fine.ent_id[s * nf + f];
    if (!claimed[id]) {
      claimed[id] = 1;
      v |= TRANSFER_OWNER;
    }
  };
  for (size_t q = 0; q < T.ident_fine.size(); ++q)
    for (int c = 0; c <= kf; ++c)
      for (int b = 0; b <= kf; ++b)
        for (int a = 0; a <= kf; ++a) visit(T.ident_fine[q], a, b, c);
  const int64_t nr = static_cast<int64_t>(T.refined_coarse.size());
  for (int64_t r = 0; r < nr; ++r)
    for (int L = 0; L <= 2 * kf; ++L)
      for (int J = 0; J <= 2 * kf; ++J)
        for (int I = 0; I <= 2 * kf; ++I) {
          const int cx = I >= kf, cy = J >= kf, cz = L >= kf;
          visit(T.refined_fine[(cx + 2 * cy + 4 * cz) * nr + r], I - cx * kf, J - cy * kf, L - cz * kf);
        }
  for (int64_t e = 0; e < fine.n_entities; ++e)  // (entities without DoFs, e.g. edges at k = 1, need none)
    MFMG_REQUIRE(count[e] == 0 || fine.ent_size[e] == 0 || claimed[e], MFMG_ERR_INVALID_ARG,
                 "transfer entity without an owner");
  return T;
}

EntityIndex::EntityIndex(const LevelDofs& active) {
  by_key.reserve(active.ent_key.size() * 2);
  for (size_t e = 0; e < active.ent_key.size(); ++e)
    if (active.ent_first[e] >= 0) by_key.emplace(active.ent_key[e], static_cast<int32_t>(e));
}

void ls_copy_pairs(const LevelDofs& H, const LevelDofs& A, const EntityIndex& index, std::vector<int32_t>& cl,
                   std::vector<int32_t>& ca) {
  cl.clear();
  ca.clear();
  MFMG_REQUIRE(H.ent_on_leaf.size() == H.ent_key.size() && H.ent_edge.size() == H.ent_key.size(),
               MFMG_ERR_INVALID_ARG, "copy map: not a local-smoothing level");
  for (size_t e = 0; e < H.ent_key.size(); ++e) {
    if (H.ent_first[e] < 0 || !H.ent_on_leaf[e] || H.ent_edge[e]) continue;
    auto it = index.by_key.find(H.ent_key[e]);
    MFMG_REQUIRE(it != index.by_key.end() && A.ent_size[it->second] == H.ent_size[e], MFMG_ERR_INVALID_ARG,
                 "copy map: level entity without an active counterpart");
    for (int t = 0; t < H.ent_size[e]; ++t) {
      cl.push_back(H.ent_first[e] + t);
      ca.push_back(A.ent_first[it->second] + t);
    }
  }
}

namespace {
// apply the hanging-node interpolation (or its transpose) to a cell vector
void apply_constraints_host(std::vector<double>& u, uint32_t m, const Tables1D& t, bool transpose) {
  const int n = t.n, k = t.k;
  std::vector<double> line(n), out(n);
  for (int d = 0; d < 3; ++d) {
    const int sd = mask_sub(m, d);
    const std::vector<double>& H = t.H[sd];
    for (int q = 0; q < n; ++q)
      for (int p = 0; p < n; ++p) {
        if (!hanging_line(m, d, p, q, k)) continue;
        auto idx = [&](int r) {
          int a = d == 0 ? r : p, b = d == 0 ? p : d == 1 ? r : q, c = d == 2 ? r : q;
          return a + n * b + n * n * c;
        };
        for (int r = 0; r < n; ++r) line[r] = u[idx(r)];
        for (int r = 0; r < n; ++r) {
          double s = 0;
          for (int r2 = 0; r2 < n; ++r2) s += transpose ? H[r2 * n + r] * line[r2] : H[r * n + r2] * line[r2];
          out[r] = s;
        }
        for (int r = 0; r < n; ++r) u[idx(r)] = out[r];
      }
  }
}
}  // namespace

// Element matrix of a mapped cell: Gauss (k+1)^3 quadrature of
// c_e (w |det J| J^{-1} J^{-T}) grad_xi phi_i . grad_xi phi_j.
static void mapped_element_matrix(const Cell& cell, uint32_t m, const Tables1D& t, const std::vector<double>& geo,
                                  int n0, std::vector<double>& Ae) {
  const int n = t.n, n3 = n * n * n;
  std::vector<double> V(n * n), Dv(n * n);  // GLL basis and derivative at the Gauss points
  for (int q = 0; q < n; ++q)
    for (int i = 0; i < n; ++i) {
      V[q * n + i] = lagrange(t.nodes, i, t.qp[q]);
      Dv[q * n + i] = lagrange_deriv(t.nodes, i, t.qp[q]);
    }
  const int l = cell.level;
  const int64_t I = cell.i >> l, J = cell.j >> l, K = cell.k >> l;
  const double* A = &geo[(I + n0 * (J + static_cast<int64_t>(n0) * K)) * 24];
  const double sc = std::ldexp(1.0, -l), coef = static_cast<double>(mask_coef(m));
  std::fill(Ae.begin(), Ae.end(), 0.0);
  std::vector<double> g(static_cast<size_t>(n3) * 3);
  for (int qc = 0; qc < n; ++qc)
    for (int qb = 0; qb < n; ++qb)
      for (int qa = 0; qa < n; ++qa) {
        double Jm[3][3], G[6];
        geo_jacobian<double>(A, (cell.i - (I << l) + t.qp[qa]) * sc, (cell.j - (J << l) + t.qp[qb]) * sc,
                             (cell.k - (K << l) + t.qp[qc]) * sc, Jm);
        for (int d = 0; d < 3; ++d)
          for (int e = 0; e < 3; ++e) Jm[d][e] *= sc;
        geo_metric<double>(Jm, coef * t.qw[qa] * t.qw[qb] * t.qw[qc], G);
        const double Gf[3][3] = {{G[0], G[1], G[2]}, {G[1], G[3], G[4]}, {G[2], G[4], G[5]}};
        for (int i = 0; i < n3; ++i) {
          const int a = i % n, b = (i / n) % n, c = i / (n * n);
          g[3 * i + 0] = Dv[qa * n + a] * V[qb * n + b] * V[qc * n + c];
          g[3 * i + 1] = V[qa * n + a] * Dv[qb * n + b] * V[qc * n + c];
          g[3 * i + 2] = V[qa * n + a] * V[qb * n + b] * Dv[qc * n + c];
        }
        for (int i = 0; i < n3; ++i) {
          double Gg[3];
          for (int d = 0; d < 3; ++d) Gg[d] = Gf[d][0] * g[3 * i] + Gf[d][1] * g[3 * i + 1] + Gf[d][2] * g[3 * i + 2];
          for (int j = 0; j < n3; ++j)
            Ae[i * n3 + j] += Gg[0] * g[3 * j] + Gg[1] * g[3 * j + 1] + Gg[2] * g[3 * j + 2];
        }
      }
}

std::vector<double> assemble_dense(const LevelDofs& L, const Tables1D& t, const std::vector<double>* geo, int geo_n0) {
  const int n = t.n, k = t.k, n3 = n * n * n;
  const int64_t N = L.n_dofs;
  std::vector<double> A(static_cast<size_t>(N * N), 0.0);
  std::vector<double> Ae(static_cast<size_t>(n3) * n3), C(static_cast<size_t>(n3) * n3), col(n3),
      tmp(static_cast<size_t>(n3) * n3);
  std::vector<int64_t> dof(n3);
  for (int64_t c = 0; c < L.n_cells; ++c) {
    const uint32_t m = L.mask[c];
    const double h = L.h0 * std::ldexp(1.0, -mask_level(m)) * static_cast<double>(mask_coef(m));
    if (geo) {
      mapped_element_matrix(L.cells[c], m, t, *geo, geo_n0, Ae);
    } else {
      for (int i = 0; i < n3; ++i)
        for (int j = 0; j < n3; ++j) {
          int a = i % n, b = (i / n) % n, cc = i / (n * n);
          int a2 = j % n, b2 = (j / n) % n, c2 = j / (n * n);
          Ae[i * n3 + j] = h * (t.K[a * n + a2] * t.M[b * n + b2] * t.M[cc * n + c2] +
                                t.M[a * n + a2] * t.K[b * n + b2] * t.M[cc * n + c2] +
                                t.M[a * n + a2] * t.M[b * n + b2] * t.K[cc * n + c2]);
        }
    }
    // C (columns = constraint interpolation of unit slot vectors)
    for (int j = 0; j < n3; ++j) {
      std::fill(col.begin(), col.end(), 0.0);
      col[j] = 1.0;
      apply_constraints_host(col, m, t, false);
      for (int i = 0; i < n3; ++i) C[i * n3 + j] = col[i];
    }
    for (int i = 0; i < n3; ++i) {
      int a = i % n, b = (i / n) % n, cc = i / (n * n);
      int s = node_slot(a, b, cc, k);
      int32_t e = L.ent[s * L.n_cells + c];
      dof[i] = e < 0 ? -1 : static_cast<int64_t>(e) + node_offset(a, b, cc, k);
    }
    // tmp = Ae C ; local = C^T tmp
    for (int i = 0; i < n3; ++i)
      for (int j = 0; j < n3; ++j) {
        double s = 0;
        for (int q = 0; q < n3; ++q) s += Ae[i * n3 + q] * C[q * n3 + j];
        tmp[i * n3 + j] = s;
      }
    for (int i = 0; i < n3; ++i) {
      if (dof[i] < 0) continue;
      for (int j = 0; j < n3; ++j) {
        if (dof[j] < 0) continue;
        double s = 0;
        for (int q = 0; q < n3; ++q) s += C[q * n3 + i] * tmp[q * n3 + j];
        A[dof[i] * N + dof[j]] += s;
      }
    }
  }
  return A;
}

}  // namespace mfmg
