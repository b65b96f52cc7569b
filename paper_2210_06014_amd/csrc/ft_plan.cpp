// Host side of a plan: validation, per-mode sort into CSR, work lists for the
// factor, combine and segment kernels, and the upload to device memory.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <thread>

#include "ft_internal.h"

namespace ft {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
ft_status fail(ft_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}
const char* last_error() { return g_last_error.c_str(); }

static int num_threads() {
  unsigned h = std::thread::hardware_concurrency();
  if (h == 0) h = 1;
  if (h > 32) h = 32;
  return (int)h;
}

template <class F>
static void parallel_for(int T, F f) {
  if (T <= 1) {
    f(0);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T);
  for (int t = 0; t < T; ++t) th.emplace_back(f, t);
  for (auto& x : th) x.join();
}

static int bits_for(int64_t n) {
  int b = 0;
  while (((int64_t)1 << b) < n) ++b;
  return b;
}

// Stable LSD radix sort of `order` (a permutation of 0..n-1) by key[order[j]].
static void radix_by_column(const int32_t* key, int64_t dim, std::vector<uint32_t>& order,
                            std::vector<uint32_t>& tmp, int T) {
  const int64_t n = (int64_t)order.size();
  int bits = bits_for(dim);
  if (bits == 0) return;
  int passes = (bits + 11) / 12;
  int digit = (bits + passes - 1) / passes;
  const int64_t B = (int64_t)1 << digit;
  std::vector<int64_t> hist((size_t)T * B);
  const int64_t per = (n + T - 1) / T;
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = pass * digit;
    const uint32_t mask = (uint32_t)(B - 1);
    const uint32_t* src = order.data();
    uint32_t* dst = tmp.data();
    parallel_for(T, [&](int t) {
      int64_t* h = hist.data() + (size_t)t * B;
      std::fill(h, h + B, 0);
      int64_t lo = t * per, hi = std::min(n, lo + per);
      for (int64_t j = lo; j < hi; ++j) ++h[((uint32_t)key[src[j]] >> shift) & mask];
    });
    int64_t run = 0;
    for (int64_t d = 0; d < B; ++d)
      for (int t = 0; t < T; ++t) {
        int64_t c = hist[(size_t)t * B + d];
        hist[(size_t)t * B + d] = run;
        run += c;
      }
    parallel_for(T, [&](int t) {
      int64_t* h = hist.data() + (size_t)t * B;
      int64_t lo = t * per, hi = std::min(n, lo + per);
      for (int64_t j = lo; j < hi; ++j) {
        uint32_t v = src[j];
        dst[h[((uint32_t)key[v] >> shift) & mask]++] = v;
      }
    });
    order.swap(tmp);
  }
}

// share g per fiber when fibers hold 4 elements or more on average: per
// element, reading g saves about a quarter of the cost of forming it per
// fiber (measured on MI355X with the Netflix-shaped workload)
static bool fiber_share(uint32_t flags, int64_t n_fibers, int64_t nnz) {
  return !(flags & (FT_NO_FIBER_SHARE | FT_NO_C_CACHE)) && n_fibers > 0 && n_fibers * 4 <= nnz &&
         n_fibers <= 0x7FFFFFFF;
}

static void pad4(std::vector<FItem>& v, int32_t kind) {
  while (v.size() % 4) v.push_back(FItem{0, 0, 0, 0, kind});
}

static ft_status build_mode(ft_plan* P, int m, const int32_t* coords, const float* vals, int T) {
  const int N = P->N;
  const int64_t nnz = P->nnz;
  const int64_t I = P->desc.dims[m];
  ModeHost& H = P->host[m];
  ModeMeta& M = P->meta[m];
  M.I = I;
  try {
    std::vector<uint32_t> order((size_t)nnz), tmp((size_t)nnz);
    for (int64_t j = 0; j < nnz; ++j) order[j] = (uint32_t)j;
    // least significant first: i_{m-1}, ..., i_{m+1} (this is the order of the
    // mode-m fibers), then i_m
    for (int k = N - 1; k >= 1; --k) {
      int n = (m + k) % N;
      radix_by_column(coords + (int64_t)n * nnz, P->desc.dims[n], order, tmp, T);
    }
    // fibers: runs of equal (i_{m+1}, ..., i_{m-1}) in the current order
    std::vector<uint32_t> fid_of((size_t)nnz);
    {
      const int64_t per = (nnz + T - 1) / T;
      std::vector<int64_t> starts((size_t)T + 1, 0);
      auto is_start = [&](int64_t j) {
        if (j == 0) return true;
        const uint32_t x = order[j], y = order[j - 1];
        for (int k = 1; k < N; ++k) {
          const int64_t base = (int64_t)((m + k) % N) * nnz;
          if (coords[base + x] != coords[base + y]) return true;
        }
        return false;
      };
      parallel_for(T, [&](int t) {
        int64_t lo = t * per, hi = std::min(nnz, lo + per), c = 0;
        for (int64_t j = lo; j < hi; ++j) c += is_start(j);
        starts[t + 1] = c;
      });
      for (int t = 0; t < T; ++t) starts[t + 1] += starts[t];
      const int64_t nfib = starts[T];
      H.fib_idx.assign((size_t)(N - 1) * nfib, 0);
      parallel_for(T, [&](int t) {
        int64_t lo = t * per, hi = std::min(nnz, lo + per), f = starts[t] - 1;
        for (int64_t j = lo; j < hi; ++j) {
          if (is_start(j)) {
            ++f;
            for (int k = 1; k < N; ++k)
              H.fib_idx[(size_t)(k - 1) * nfib + f] = coords[(int64_t)((m + k) % N) * nnz + order[j]];
          }
          fid_of[order[j]] = (uint32_t)f;
        }
      });
      P->meta[m].n_fibers = nfib;
    }
    radix_by_column(coords + (int64_t)m * nnz, P->desc.dims[m], order, tmp, T);
    tmp.clear();
    tmp.shrink_to_fit();
    H.row_ptr.assign((size_t)I + 1, 0);
    const int32_t* im = coords + (int64_t)m * nnz;
    for (int64_t j = 0; j < nnz; ++j) ++H.row_ptr[(size_t)im[j] + 1];
    for (int64_t i = 0; i < I; ++i) H.row_ptr[i + 1] += H.row_ptr[i];
    H.idx.resize((size_t)(N - 1) * nnz);
    H.val.resize((size_t)nnz);
    H.perm.resize((size_t)nnz);
    H.fid.resize((size_t)nnz);
    const int64_t per = (nnz + T - 1) / T;
    parallel_for(T, [&](int t) {
      int64_t lo = t * per, hi = std::min(nnz, lo + per);
      for (int64_t p = lo; p < hi; ++p) {
        uint32_t x = order[p];
        for (int k = 1; k < N; ++k) H.idx[(size_t)(k - 1) * nnz + p] = coords[(int64_t)((m + k) % N) * nnz + x];
        H.val[p] = vals[x];
        H.perm[p] = x;
        H.fid[p] = (int32_t)fid_of[x];
      }
    });
  } catch (const std::bad_alloc&) {
    return fail(FT_ERR_NOMEM, "host allocation failed while sorting mode " + std::to_string(m));
  }

  // FT_RELAXED: a row longer than the head is dealt in stride order
  // (Q = ceil(L / head): positions 0, Q, 2Q, ..., then 1, 1 + Q, ...) so that
  // its head and each chunk hold a sample of the whole row rather than a
  // narrow slice of the sorted order.  Only the factor passes depend on the
  // order within a row, so they read a dealt copy of the indices and values
  // (fidx, fval) and the fiber ids (read by nothing else) are dealt in place;
  // the core, loss and gradient passes keep the sorted arrays, whose
  // neighbouring elements share the next mode's index (cache locality of the
  // gathers).
  // head length of this mode: the plan's, or (exact plans by default) the
  // longest of 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32 chunks, up to the
  // plan's cap, that passes two tests.
  //  * Not above L_q, the row length reached by the longest rows holding a
  //    quarter of the mode's elements.  Those rows then still split into
  //    chunk maps, which run beside their heads; a head as long as such a row
  //    would leave it one slow serial chain (rows of 10000 elements at order
  //    4: 36 ms per iteration with head 8192, 52 ms with 16384).  Zipf rows
  //    give L_q far above the cap.
  //  * The serial chain of a head must not outlast the rest of the launch.
  //    With S(h) elements on in-place chains and M(h) in chunk maps, the
  //    launch costs about t_m (r_s S + M) and a head of h elements a h, so
  //    the test is r_a h <= 0.8 (r_s S + M), r_a = a / t_m and r_s = t_s /
  //    t_m.  A chain step forms g (J R FMAs on 16 lanes) unless the mode
  //    shares g per fiber; a map step adds the J x J update.  Fitted to
  //    MI355X launch times of the Netflix-shaped tensors and the 1000^3
  //    density tensors: r_a = 2358 (J = 32), 3100 (J = 16) with g formed per
  //    step, 1200 and 2000 with g read; r_s = 0.5 and 0.2 / 0.3.  This is
  //    what shortens the heads of tensors with few long rows (1000 rows of
  //    20000 elements: 5120 instead of 16384, 2.2 instead of 4.8 ms per pass).
  M.head = P->head;
  if (M.head == 0) {
    std::vector<int64_t> lens;
    lens.reserve((size_t)I);
    for (int64_t i = 0; i < I; ++i)
      if (H.row_ptr[i + 1] > H.row_ptr[i]) lens.push_back(H.row_ptr[i + 1] - H.row_ptr[i]);
    std::sort(lens.begin(), lens.end(), std::greater<int64_t>());
    int64_t acc = 0, lq = 0;
    for (int64_t L : lens) {
      acc += L;
      lq = L;
      if (4 * acc >= nnz) break;
    }
    const bool shares_g = fiber_share(P->desc.flags, M.n_fibers, nnz);
    const double ra = P->J >= 32 ? (shares_g ? 1200.0 : 2358.0) : (shares_g ? 2000.0 : 3100.0);
    const double rs = shares_g ? (P->J >= 32 ? 0.2 : 0.3) : 0.5;
    const int64_t maxL = lens.empty() ? 0 : lens[0];
    static const int kChunks[] = {2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32};
    int64_t h = 2 * P->chunk;
    for (int k : kChunks) {
      const int64_t c = (int64_t)k * P->chunk;
      if (k == 2) continue;
      if (c > P->head_cap || c > lq) break;
      double S = 0.0, Mm = 0.0;
      for (int64_t L : lens) {
        S += (double)std::min(L, c);
        Mm += (double)std::max<int64_t>(L - c, 0);
      }
      if (ra * (double)std::min(c, maxL) > 0.8 * (rs * S + Mm)) break;
      h = c;
    }
    M.head = h;
  }
  if (P->relaxed && M.head > 0) {
    const int64_t hl0 = M.head;
    int64_t maxL = 0;
    for (int64_t i = 0; i < I; ++i) maxL = std::max(maxL, H.row_ptr[i + 1] - H.row_ptr[i]);
    if (maxL > hl0) {
      try {
        H.fidx = H.idx;
        H.fval = H.val;
        H.fperm = H.perm;
        std::vector<int64_t> src((size_t)maxL);
        std::vector<int32_t> t32((size_t)maxL);
        std::vector<int64_t> t64((size_t)maxL);
        std::vector<float> tf((size_t)maxL);
        auto deal = [&](auto* base, auto& tmp, int64_t s, int64_t L) {
          for (int64_t t = 0; t < L; ++t) tmp[t] = base[s + src[t]];
          for (int64_t t = 0; t < L; ++t) base[s + t] = tmp[t];
        };
        for (int64_t i = 0; i < I; ++i) {
          const int64_t s = H.row_ptr[i], L = H.row_ptr[i + 1] - s;
          if (L <= hl0) continue;
          const int64_t Q = (L + hl0 - 1) / hl0;
          int64_t o = 0;
          for (int64_t r = 0; r < Q; ++r)
            for (int64_t t = r; t < L; t += Q) src[o++] = t;
          for (int k = 0; k < N - 1; ++k) deal(H.fidx.data() + (int64_t)k * nnz, t32, s, L);
          deal(H.fval.data(), tf, s, L);
          deal(H.fperm.data(), t64, s, L);
          if (!H.fid.empty()) deal(H.fid.data(), t32, s, L);
        }
      } catch (const std::bad_alloc&) {
        return fail(FT_ERR_NOMEM, "host allocation failed while dealing mode " + std::to_string(m));
      }
    }
  }

  // factor work lists: a row of at most `head` elements is one serial item;
  // a longer row is a head item (its first `head` elements, updated in
  // place) followed by chunk items whose maps the combine applies in order
  const int64_t chunk = P->chunk, hl = M.head;
  std::vector<FItem> light, head;
  int64_t n_heavy = 0, n_maps = 0, max_row = 0, nonempty = 0;
  std::vector<int64_t> heavy_rows, heavy_base, heavy_nmaps;
  for (int64_t i = 0; i < I; ++i) {
    int64_t s = H.row_ptr[i], L = H.row_ptr[i + 1] - s;
    if (L == 0) continue;
    ++nonempty;
    max_row = std::max(max_row, L);
    if (L <= hl) {
      light.push_back(FItem{s, (int32_t)L, (int32_t)i, 0, ITEM_LIGHT});
      continue;
    }
    const int64_t K = (L - hl + chunk - 1) / chunk;  // chunk maps after the head
    head.push_back(FItem{s, (int32_t)hl, (int32_t)i, (int32_t)n_heavy, ITEM_HEAD});
    heavy_rows.push_back(i);
    heavy_base.push_back(n_maps);
    heavy_nmaps.push_back(K);
    for (int64_t c = 0; c < K; ++c) {
      const int64_t st = s + hl + c * chunk;
      H.compose.push_back(FItem{st, (int32_t)std::min(chunk, L - hl - c * chunk), (int32_t)i, (int32_t)(n_maps + c),
                                ITEM_COMPOSE});
    }
    n_maps += K;
    ++n_heavy;
  }
  if (n_maps > 0x7FFFFFFF || n_heavy > 0x7FFFFFFF) return fail(FT_ERR_SHAPE, "too many chunks");
  std::stable_sort(H.compose.begin(), H.compose.end(), [](const FItem& a, const FItem& b) { return a.len > b.len; });
  std::stable_sort(light.begin(), light.end(), [](const FItem& a, const FItem& b) { return a.len > b.len; });
  pad4(H.compose, ITEM_COMPOSE);
  H.apply = head;
  pad4(H.apply, ITEM_HEAD);
  H.apply.insert(H.apply.end(), light.begin(), light.end());
  pad4(H.apply, ITEM_LIGHT);

  // combine levels: a heavy row whose maps number at most fanin has them
  // applied in sequence to its head vector (a final item); a longer row first
  // has groups of `fanin` consecutive maps folded into one, level by level.
  // Each level lists its folds first, then its final items by descending map
  // count (similar counts share a wavefront).
  const int64_t fan = P->fanin, fin = P->fanin;
  std::vector<int64_t> cur_off(heavy_base), cur_n(heavy_nmaps);
  int64_t region_base[2] = {0, n_maps};
  int level = 0;
  int64_t out0 = 0;
  std::vector<int64_t> active;
  for (int64_t h = 0; h < n_heavy; ++h) active.push_back(h);
  while (!active.empty()) {
    std::vector<CItem> items, finals;
    std::vector<int64_t> next;
    int64_t out_next = 0;
    int dst = (level + 1) & 1;
    for (int64_t h : active) {
      int64_t n = cur_n[h], off = cur_off[h];
      if (n <= fin) {
        finals.push_back(CItem{off, -1, (int32_t)n, (int32_t)heavy_rows[h], (int32_t)h, 0});
        continue;
      }
      int64_t groups = (n + fan - 1) / fan;
      int64_t base = region_base[dst] + out_next;
      for (int64_t g = 0; g < groups; ++g)
        items.push_back(CItem{off + g * fan, base + g, (int32_t)std::min(fan, n - g * fan), (int32_t)heavy_rows[h],
                              (int32_t)h, 0});
      out_next += groups;
      cur_off[h] = base;
      cur_n[h] = groups;
      next.push_back(h);
    }
    if (level == 0) out0 = out_next;
    if (out_next > (dst == 1 ? INT64_MAX : n_maps)) return fail(FT_ERR_STATE, "combine plan overflow");
    std::stable_sort(finals.begin(), finals.end(), [](const CItem& x, const CItem& y) { return x.count > y.count; });
    M.level_ncomp.push_back((int64_t)items.size());
    items.insert(items.end(), finals.begin(), finals.end());
    H.levels.push_back(std::move(items));
    active.swap(next);
    ++level;
  }

  // relaxed merge items: a heavy row's chunk increments are slots
  // heavy_base .. heavy_base + K - 1, in row order.  Level 1 sums groups of
  // kRelaxGroup consecutive slots of one row into group records; level 2 sums
  // a row's group records (consecutive) and updates the row.  Larger rows first.
  if (P->relaxed) {
    std::vector<CItem> merges;
    int64_t n_groups = 0;
    for (int64_t h = 0; h < n_heavy; ++h) {
      const int64_t i = heavy_rows[h], L = H.row_ptr[i + 1] - H.row_ptr[i], K = heavy_nmaps[h];
      const int64_t ng = (K + kRelaxGroup - 1) / kRelaxGroup;
      for (int64_t g = 0; g < ng; ++g)
        H.relax.push_back(CItem{heavy_base[h] + g * kRelaxGroup, n_groups + g,
                                (int32_t)std::min<int64_t>(kRelaxGroup, K - g * kRelaxGroup), (int32_t)i,
                                (int32_t)h, 0});
      merges.push_back(CItem{n_groups, L - hl, (int32_t)ng, (int32_t)i, (int32_t)h, 0});
      n_groups += ng;
    }
    std::stable_sort(H.relax.begin(), H.relax.end(), [](const CItem& x, const CItem& y) { return x.count > y.count; });
    std::stable_sort(merges.begin(), merges.end(), [](const CItem& x, const CItem& y) { return x.count > y.count; });
    M.n_relax_groups = n_groups;
    H.relax.insert(H.relax.end(), merges.begin(), merges.end());
  }

  // segments for the core, loss and gradient passes
  H.seg_ptr.assign((size_t)I + 1, 0);
  for (int64_t i = 0; i < I; ++i) {
    int64_t s = H.row_ptr[i], L = H.row_ptr[i + 1] - s;
    for (int64_t o = 0; o < L; o += kSegLen)
      H.segs.push_back(Seg{s + o, (int32_t)std::min<int64_t>(kSegLen, L - o), (int32_t)i});
    H.seg_ptr[i + 1] = (int64_t)H.segs.size();
  }

  // runs of equal column-0 index (mode m + 1) within rows: the segment
  // passes gather that C row once per run
  {
    int64_t runs = 0;
    const int32_t* c0 = H.idx.data();
    for (int64_t i = 0; i < I; ++i)
      for (int64_t p = H.row_ptr[i]; p < H.row_ptr[i + 1]; ++p) runs += (p == H.row_ptr[i] || c0[p] != c0[p - 1]);
    M.n_runs = runs;
  }

  M.use_fiber = fiber_share(P->desc.flags, M.n_fibers, nnz);
  if (!M.use_fiber) {
    H.fid.clear();
    H.fid.shrink_to_fit();
    H.fib_idx.clear();
    H.fib_idx.shrink_to_fit();
  }
  M.n_compose = (int64_t)H.compose.size();
  M.n_apply = (int64_t)H.apply.size();
  M.n_heavy = n_heavy;
  M.n_maps = n_maps;
  M.n_level_out0 = out0;
  M.n_segs = (int64_t)H.segs.size();
  M.n_relax = (int64_t)H.relax.size() - M.n_relax_groups;
  int64_t off = 0;
  for (auto& L : H.levels) {
    M.level_off.push_back(off);
    M.level_len.push_back((int64_t)L.size());
    off += (int64_t)L.size();
  }
  ft_mode_info& inf = M.info;
  inf.rows = I;
  inf.nonempty_rows = nonempty;
  inf.max_row = max_row;
  inf.light_rows = (int64_t)light.size();
  inf.heavy_rows = n_heavy;
  inf.chunks = (int64_t)head.size() + n_maps;
  inf.segments = M.n_segs;
  inf.combine_levels = (int32_t)H.levels.size();
  inf.fibers = M.n_fibers;
  inf.fiber_shared = M.use_fiber ? 1 : 0;
  inf.head = (int32_t)M.head;
  inf.chunk = P->chunk;
  inf.runs = M.n_runs;
  return FT_OK;
}

// Offsets of the plan's device arrays in the caller's workspace, and the
// scratch layout every parameter set brings (sized for the largest mode).
static void layout(ft_plan* P) {
  const int N = P->N, J = P->J, R = P->R;
  const bool perm = (P->desc.flags & FT_WITH_PERM) != 0;
  Layout L;
  P->off.assign(N, ModeOff{});
  int64_t max_slots = 1, max_heavy = 1, max_segs = 1, max_fib = 0, map_floats = 0;
  for (int m = 0; m < N; ++m) {
    const ModeHost& H = P->host[m];
    const ModeMeta& M = P->meta[m];
    ModeOff& o = P->off[m];
    size_t nlev = 0;
    for (auto& v : H.levels) nlev += v.size();
    o.row_ptr = L.add(H.row_ptr.size() * sizeof(int64_t));
    o.idx = L.add(H.idx.size() * sizeof(int32_t));
    o.val = L.add(H.val.size() * sizeof(float));
    o.perm = L.add(perm ? H.perm.size() * sizeof(int32_t) : 0);
    o.compose = L.add(H.compose.size() * sizeof(FItem));
    o.apply = L.add(H.apply.size() * sizeof(FItem));
    o.levels = L.add(nlev * sizeof(CItem));
    o.relax = L.add(P->relaxed ? H.relax.size() * sizeof(CItem) : 0);
    o.segs = L.add(H.segs.size() * sizeof(Seg));
    o.seg_ptr = L.add(H.seg_ptr.size() * sizeof(int64_t));
    o.fid = L.add(M.use_fiber ? H.fid.size() * sizeof(int32_t) : 0);
    o.fidx = L.add(H.fidx.size() * sizeof(int32_t));
    o.fval = L.add(H.fval.size() * sizeof(float));
    o.fib_idx = L.add(M.use_fiber ? H.fib_idx.size() * sizeof(int32_t) : 0);
    if (M.use_fiber) max_fib = std::max(max_fib, M.n_fibers);
    max_slots = std::max(max_slots, M.n_maps + M.n_level_out0);
    max_heavy = std::max(max_heavy, M.n_heavy);
    max_segs = std::max(max_segs, M.n_segs);
    map_floats = std::max(map_floats, max_slots * (J * J + J));
    if (P->relaxed)
      map_floats = std::max(map_floats, relax_incr_floats(M.n_maps, J) + 2 * M.n_relax_groups * (J + 1));
  }
  P->device_bytes = L.bytes;
  Layout S;
  ScratchOff& so = P->soff;
  so.maps = S.add((size_t)std::max<int64_t>(map_floats, 1) * sizeof(float));
  so.map_scale = S.add((size_t)max_slots * sizeof(double));
  so.hvec = S.add((size_t)max_heavy * J * sizeof(float));
  so.partials = S.add((size_t)(kPartials + kPartials / 32 + 1) * J * R * sizeof(float));
  so.dpartials = S.add(((size_t)kPartials + 2 * FT_MAX_ORDER * 256) * sizeof(double));
  so.tseg = S.add((size_t)max_segs * R * sizeof(float));
  so.gfib = S.add((size_t)max_fib * J * sizeof(float));
  P->scratch_bytes = S.bytes;
}

template <class T>
static T* at(void* base, size_t off) {
  return off == SIZE_MAX ? nullptr : reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

Scratch scratch_of(const ft_plan* P, const ft_params* p) {
  Scratch S;
  const ScratchOff& o = P->soff;
  S.maps = at<float>(p->scratch, o.maps);
  S.map_scale = at<double>(p->scratch, o.map_scale);
  S.hvec = at<float>(p->scratch, o.hvec);
  S.partials = at<float>(p->scratch, o.partials);
  S.dpartials = at<double>(p->scratch, o.dpartials);
  S.tseg = at<float>(p->scratch, o.tseg);
  S.gfib = at<float>(p->scratch, o.gfib);
  return S;
}

}  // namespace ft

using namespace ft;

extern "C" ft_status ft_plan_create(ft_plan** out, const ft_desc* d, const int32_t* coords, const float* vals) {
  if (!out || !d) return fail(FT_ERR_ARG, "null argument");
  *out = nullptr;
  if (d->order < 2 || d->order > FT_MAX_ORDER) return fail(FT_ERR_SHAPE, "order must be in 2..FT_MAX_ORDER");
  if (d->nnz < 0 || d->nnz > (int64_t)0xFFFFFFFFLL) return fail(FT_ERR_SHAPE, "nnz out of range");
  if (d->nnz > 0 && (!coords || !vals)) return fail(FT_ERR_ARG, "null coords or vals");
  if (d->R < 1) return fail(FT_ERR_SHAPE, "R must be positive");
  for (int n = 0; n < d->order; ++n) {
    if (d->dims[n] < 1 || d->dims[n] > 0x7FFFFFFF) return fail(FT_ERR_SHAPE, "dimension out of range");
    if (d->J[n] != d->J[0]) return fail(FT_ERR_UNSUPPORTED, "all J_n must be equal");
  }
  // the kernels gather C rows by 32-bit byte offsets from the table's base
  for (int n = 0; n < d->order; ++n)
    if (d->dims[n] * (int64_t)d->R * 4 >= ((int64_t)1 << 31))
      return fail(FT_ERR_SHAPE, "mode " + std::to_string(n) + ": I_n * R * 4 bytes must be below 2^31");
  if (!supported(d->order, d->J[0], d->R))
    return fail(FT_ERR_UNSUPPORTED, "no kernels compiled for order " + std::to_string(d->order) + ", J " +
                                        std::to_string(d->J[0]) + ", R " + std::to_string(d->R));
  if (d->chunk < 0 || d->head < 0 || d->fanin < 0 || d->fanin == 1)
    return fail(FT_ERR_ARG, "bad chunk, head or fanin");
  if ((d->flags & FT_NO_C_CACHE) && !(d->order == 3 && d->J[0] == 16 && d->R == 16))
    return fail(FT_ERR_UNSUPPORTED, "FT_NO_C_CACHE is built for order 3 with J = R = 16 only");
  if ((d->flags & FT_RELAXED) && (d->flags & FT_NO_C_CACHE))
    return fail(FT_ERR_UNSUPPORTED, "FT_RELAXED is not built with FT_NO_C_CACHE");
  if ((d->flags & FT_WITH_PERM) && d->nnz > 0x7FFFFFFF) return fail(FT_ERR_SHAPE, "FT_WITH_PERM needs nnz < 2^31");
  const int N = d->order;
  const int64_t nnz = d->nnz;
  const int T = num_threads();
  // index validation
  std::atomic<int64_t> bad{-1};
  {
    const int64_t total = (int64_t)N * nnz, per = (total + T - 1) / T;
    parallel_for(T, [&](int t) {
      int64_t lo = t * per, hi = std::min(total, lo + per);
      for (int64_t k = lo; k < hi; ++k) {
        int64_t n = k / (nnz > 0 ? nnz : 1);
        int32_t c = coords[k];
        if (c < 0 || c >= d->dims[n]) {
          bad.store(k);
          return;
        }
      }
    });
  }
  if (bad.load() >= 0) {
    int64_t k = bad.load();
    return fail(FT_ERR_INDEX, "coordinate out of range: mode " + std::to_string(k / nnz) + ", element " +
                                  std::to_string(k % nnz) + ", value " + std::to_string(coords[k]));
  }
  ft_plan* P = new (std::nothrow) ft_plan();
  if (!P) return fail(FT_ERR_NOMEM, "plan allocation failed");
  P->desc = *d;
  P->N = N;
  P->J = d->J[0];
  P->R = d->R;
  P->nnz = nnz;
  // Default piece lengths.  Exact passes: a chunk map costs 4 J^2 flops per
  // element and a fold of maps J^3, while the serial in-place chains run
  // beside the maps in the same launch, so with J >= 32 longer chunks and
  // far longer heads pay (measured on MI355X with the Netflix-shaped tensor:
  // 32.7 ms per iteration with chunk 512 and head 1024, 26.7 with chunk 1024
  // and head 24576); J = 16 gains less (11.4 ms with head 4096, 11.0 with
  // 12288).  Each mode picks its head up to the cap (32 chunks at J >= 32,
  // 24 at J = 16, 2 below) from its row lengths, as build_mode describes.
  // Relaxed passes keep chunk 512 and head 1024: their chunks start from the
  // head's result, so a long head is serial time, and the chunk length is
  // part of the semantics.
  const int J0 = d->J[0];
  const bool rlx = (d->flags & FT_RELAXED) != 0;
  const int long_heads = rlx ? 2 : J0 >= 32 ? 32 : J0 >= 16 ? 24 : 2;
  P->chunk = d->chunk ? d->chunk : (!rlx && J0 >= 32 ? 1024 : 512);
  // an explicit head, the relaxed default, or 0: each mode picks its own up to head_cap
  P->head = d->head ? d->head : rlx ? 2 * P->chunk : 0;
  P->head_cap = (int64_t)P->chunk * long_heads;
  P->no_c_cache = (d->flags & FT_NO_C_CACHE) != 0;
  P->relaxed = (d->flags & FT_RELAXED) != 0;
  P->fused = !(d->flags & FT_SPLIT_FACTOR);
  P->run_reuse = (d->flags & FT_RUN_REUSE) && N >= 3;
  P->fanin = std::min(d->fanin ? d->fanin : max_fanin(d->J[0]), max_fanin(d->J[0]));
  try {
    P->meta.resize(N);
    P->host.resize(N);
    P->dev.resize(N);
  } catch (const std::bad_alloc&) {
    delete P;
    return fail(FT_ERR_NOMEM, "plan allocation failed");
  }
  for (int m = 0; m < N; ++m) {
    ft_status s = build_mode(P, m, coords, vals, T);
    if (s != FT_OK) {
      delete P;
      return s;
    }
  }
  // the loss walks the mode with the fewest runs (longest on average)
  for (int m = 1; m < N; ++m)
    if (P->meta[m].n_runs < P->meta[P->loss_mode].n_runs) P->loss_mode = m;
  layout(P);
  P->host_valid = true;
  *out = P;
  return FT_OK;
}

namespace {
template <class T>
hipError_t copy_in(void* base, size_t off, const std::vector<T>& src, hipStream_t s) {
  if (off == SIZE_MAX || src.empty()) return hipSuccess;
  return hipMemcpyAsync(static_cast<char*>(base) + off, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}
}  // namespace

extern "C" ft_status ft_plan_query(const ft_plan* P, size_t* device_bytes, size_t* scratch_bytes) {
  if (!P) return fail(FT_ERR_ARG, "null plan");
  if (device_bytes) *device_bytes = P->device_bytes;
  if (scratch_bytes) *scratch_bytes = P->scratch_bytes;
  return FT_OK;
}

extern "C" ft_status ft_plan_upload(ft_plan* P, void* ws, size_t ws_bytes, void* stream) {
  if (!P) return fail(FT_ERR_ARG, "null plan");
  if (!P->host_valid) return fail(FT_ERR_STATE, "plan already uploaded and its host copy released");
  if (!ws || ws_bytes < P->device_bytes)
    return fail(FT_ERR_WORKSPACE, "plan workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                      std::to_string(P->device_bytes));
  if (reinterpret_cast<uintptr_t>(ws) % kAlign) return fail(FT_ERR_WORKSPACE, "plan workspace not 256-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  // the int32 permutations and the concatenated combine levels are staged
  // here and must live until the copies have completed (the wait below)
  std::vector<std::vector<int32_t>> perm32(P->N);
  std::vector<std::vector<CItem>> levels(P->N);
  for (int m = 0; m < P->N && e == hipSuccess; ++m) {
    const ModeHost& H = P->host[m];
    const ModeOff& o = P->off[m];
    if (o.perm != SIZE_MAX) perm32[m].assign(H.perm.begin(), H.perm.end());
    for (auto& L : H.levels) levels[m].insert(levels[m].end(), L.begin(), L.end());
    e = copy_in(ws, o.row_ptr, H.row_ptr, s);
    if (e == hipSuccess) e = copy_in(ws, o.idx, H.idx, s);
    if (e == hipSuccess) e = copy_in(ws, o.val, H.val, s);
    if (e == hipSuccess) e = copy_in(ws, o.perm, perm32[m], s);
    if (e == hipSuccess) e = copy_in(ws, o.compose, H.compose, s);
    if (e == hipSuccess) e = copy_in(ws, o.apply, H.apply, s);
    if (e == hipSuccess) e = copy_in(ws, o.levels, levels[m], s);
    if (e == hipSuccess) e = copy_in(ws, o.relax, H.relax, s);
    if (e == hipSuccess) e = copy_in(ws, o.segs, H.segs, s);
    if (e == hipSuccess) e = copy_in(ws, o.seg_ptr, H.seg_ptr, s);
    if (e == hipSuccess) e = copy_in(ws, o.fid, H.fid, s);
    if (e == hipSuccess) e = copy_in(ws, o.fib_idx, H.fib_idx, s);
    if (e == hipSuccess) e = copy_in(ws, o.fidx, H.fidx, s);
    if (e == hipSuccess) e = copy_in(ws, o.fval, H.fval, s);
  }
  const hipError_t w = hipStreamSynchronize(s);
  if (e == hipSuccess) e = w;
  if (e != hipSuccess) return fail(FT_ERR_HIP, std::string("plan upload failed: ") + hipGetErrorString(e));
  for (int m = 0; m < P->N; ++m) {
    const ModeOff& o = P->off[m];
    ModeDev& D = P->dev[m];
    D.row_ptr = at<int64_t>(ws, o.row_ptr);
    D.idx = at<int32_t>(ws, o.idx);
    D.val = at<float>(ws, o.val);
    D.perm = at<int32_t>(ws, o.perm);
    D.compose = at<FItem>(ws, o.compose);
    D.apply = at<FItem>(ws, o.apply);
    D.levels = at<CItem>(ws, o.levels);
    D.relax = at<CItem>(ws, o.relax);
    D.segs = at<Seg>(ws, o.segs);
    D.seg_ptr = at<int64_t>(ws, o.seg_ptr);
    D.fid = at<int32_t>(ws, o.fid);
    D.fib_idx = at<int32_t>(ws, o.fib_idx);
    D.fidx = at<int32_t>(ws, o.fidx);
    D.fval = at<float>(ws, o.fval);
  }
  P->uploaded = true;
  if (!(P->desc.flags & FT_KEEP_HOST)) {
    for (auto& H : P->host) H = ModeHost{};
    P->host_valid = false;
  }
  return FT_OK;
}

extern "C" void ft_plan_destroy(ft_plan* P) { delete P; }

extern "C" ft_status ft_plan_mode_info(const ft_plan* P, int32_t mode, ft_mode_info* info) {
  if (!P || !info) return fail(FT_ERR_ARG, "null argument");
  if (mode < 0 || mode >= P->N) return fail(FT_ERR_ARG, "mode out of range");
  *info = P->meta[mode].info;
  return FT_OK;
}

extern "C" ft_status ft_plan_host_csr(const ft_plan* P, int32_t mode, int32_t factor_order, int64_t* row_ptr,
                                      int32_t* idx, float* vals, int64_t* perm) {
  if (!P) return fail(FT_ERR_ARG, "null plan");
  if (mode < 0 || mode >= P->N) return fail(FT_ERR_ARG, "mode out of range");
  if (!P->host_valid) return fail(FT_ERR_STATE, "host plan not kept (use FT_KEEP_HOST)");
  const ModeHost& H = P->host[mode];
  const bool dealt = factor_order && !H.fidx.empty();
  const std::vector<int32_t>& I = dealt ? H.fidx : H.idx;
  const std::vector<float>& V = dealt ? H.fval : H.val;
  const std::vector<int64_t>& Pm = dealt ? H.fperm : H.perm;
  if (row_ptr) std::memcpy(row_ptr, H.row_ptr.data(), H.row_ptr.size() * sizeof(int64_t));
  if (idx && !I.empty()) std::memcpy(idx, I.data(), I.size() * sizeof(int32_t));
  if (vals && !V.empty()) std::memcpy(vals, V.data(), V.size() * sizeof(float));
  if (perm && !Pm.empty()) std::memcpy(perm, Pm.data(), Pm.size() * sizeof(int64_t));
  return FT_OK;
}
