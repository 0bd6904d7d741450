// Execution engine shared by the single-curve entry points, the batch search
// and the captured graphs: factor allocation, launch schedules of the blocked
// Cholesky and of the triangular inverse for one or more factors at once, and
// the enqueue sequences of the factorisation, the inverse, the linear search
// and the periodic search. Nothing here synchronises except run_factor when
// asked to read the statuses back.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.hpp"

namespace nu {

namespace {

int tiles_of(const GemmProblem& g, int tm, int tn) {
  const int rm = g.M / tm, rn = g.N / tn;
  return (g.flags & G_C_LOWER_TILES) ? rm * (rm + 1) / 2 : rm * rn;
}

// useful flops of a problem (zeros of triangular operands not counted)
double useful_flops(const GemmProblem& g) {
  const double M = g.M, N = g.N, K = g.K;
  if (g.flags & G_C_LOWER_TILES) return M * (M + 1) * K;          // 2 K per lower element
  if (g.flags & (G_B_LOWER | G_B_UPPER)) return M * N * (N + 1);  // triangular N x N right factor
  if (g.flags & G_A_LOWER) return N * M * (M + 1);                // triangular M x M left factor
  if ((g.flags & G_BT) && g.K == TB && g.N == TB) return M * N * (K + 1);  // panel: triangular X_kk^T
  return 2.0 * M * N * K;
}

// Append one launch's problems, numbering tiles from 0 within the launch. A
// launch with fewer 128 x 128 tiles than small_below uses 64 x 64 tiles (four
// times the workgroups, each a quarter of the work), or 64 x 128 tiles when
// its problems write C over A (N = 128 there: each tile keeps whole rows).
Range add_launch(std::vector<GemmProblem>& sched, std::vector<GemmProblem> probs, int small_below) {
  Range r;
  if (probs.empty()) return r;
  r.first = (int)sched.size();
  r.count = (int)probs.size();
  int big = 0;
  bool inplace = false;
  for (auto& p : probs) {
    big += tiles_of(p, TB, TB);
    inplace = inplace || (p.flags & G_C_IS_A);
  }
  if (big < small_below) {
    r.tile_m = 64;
    r.tile_n = inplace ? TB : 64;
  }
  int t = 0;
  for (auto& p : probs) {
    p.tiles_n = p.N / r.tile_n;
    p.tile_begin = t;
    p.tile_count = tiles_of(p, r.tile_m, r.tile_n);
    t += p.tile_count;
    r.flops += useful_flops(p);
    sched.push_back(p);
  }
  r.tiles = t;
  return r;
}

// element (row, col) of a row-major matrix with leading dimension ld and element size es
inline const void* at(const void* base, int64_t row, int64_t col, int64_t ld, size_t es) {
  return static_cast<const char*>(base) + (size_t)(row * ld + col) * es;
}
inline void* at(void* base, int64_t row, int64_t col, int64_t ld, size_t es) {
  return static_cast<char*>(base) + (size_t)(row * ld + col) * es;
}

GemmProblem prob(const void* A, int64_t lda, const void* B, int64_t ldb, void* C, int64_t ldc, int M, int N, int K,
                 int flags, double alpha, double beta) {
  GemmProblem g{};
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.flags = flags;
  g.alpha = alpha;
  g.beta = beta;
  return g;
}

struct Node {
  int a, mid, b;
};

// The root splits at 55 % of the blocks (trees of 8 blocks or more), every
// other node in the middle: the leading part, which the inverse prefetch
// starts inside the factorisation, takes a little more of the work (the
// products add up to the same flops whatever the split). At N = 18000:
// 71.0 ms per step against 71.5 with the root in the middle (45 %: 73.3,
// 60 %: 72.6-72.9).
void build_tree(int a, int b, int depth, std::vector<std::vector<Node>>& levels) {
  if (b - a < 2) return;
  const int mid = depth == 0 && b - a >= 8 ? a + (b - a) * 11 / 20 : a + (b - a + 1) / 2;
  if ((int)levels.size() <= depth) levels.resize(depth + 1);
  levels[depth].push_back({a, mid, b});
  build_tree(a, mid, depth + 1, levels);
  build_tree(mid, b, depth + 1, levels);
}

// levels of the inverse tree in execution order (deepest first)
std::vector<std::vector<Node>> inverse_levels(int nblk) {
  std::vector<std::vector<Node>> levels;
  build_tree(0, nblk, 0, levels);
  std::reverse(levels.begin(), levels.end());
  return levels;
}

// Outer panel width of the Cholesky, in TB blocks: each panel is factored
// block by block (diagonal block, its column, the update of the panel's
// remaining columns), then the trailing matrix gets one update of depth
// PANEL * TB. At N = 18000 with the inverse prefetch: 70.2-70.4 ms per step
// with 6, against 71.1-71.2 with 4, 70.6-70.8 with 5, 71.3-71.5 with 8 and
// 72.5 with 3.
constexpr int PANEL = 6;

}  // namespace

// ---------------------------------------------------------------------------
// Schedules

// The chain of a factorisation (diagonal blocks, panels, panel updates and the
// next panel's update) is latency bound, and with the lookahead and the
// inverse prefetch its workgroups share compute units with the trailing
// updates and the early inverse. Its GEMM problems carry G_PRIO (and the
// diagonal-block kernel raises its own priority), so their waves issue first on
// a shared CU: at N = 18000, 63.1-63.4 -> 62.5-62.7 ms per step, outputs
// bitwise unchanged.
void plan_cholesky(const std::vector<nu_factor*>& Fs, const Tuning& tu, Plan& P) {
  int steps = 0;
  for (auto* F : Fs) steps = std::max(steps, F->nblk);
  P.panel.assign(steps, Range());
  P.pupd.assign(steps, Range());
  P.next.assign(steps, Range());
  P.rest.assign(steps, Range());
  P.job_first.assign(steps, 0);
  P.job_count.assign(steps, 0);
  const size_t es = sizeof(double);
  for (int k = 0; k < steps; ++k) {
    P.job_first[k] = (int)P.jobs.size();
    std::vector<GemmProblem> pan, pup, nx, rs;
    for (auto* F : Fs) {
      if (k >= F->nblk) continue;
      const int64_t np = F->np;
      const int64_t off = (int64_t)k * TB;
      P.jobs.push_back(PotrfJob{F->L, F->X, F->parts(), F->status_dev(), np, off, k, 0});
      const int p0 = k / PANEL * PANEL;
      const int pw = std::min(PANEL, F->nblk - p0);
      const int rest = (int)(np - off - TB);
      if (rest > 0) {
        void* col = at(F->L, off + TB, off, np, es);  // rows below the diagonal block, block column k
        const void* xkk = at(F->X, off, off, np, es);
        pan.push_back(prob(col, np, xkk, np, col, np, rest, TB, TB, G_BT | G_C_IS_A | G_PRIO, 1.0, 0.0));
        const int inner = (p0 + pw - k - 1) * TB;  // columns of this panel right of block k
        if (inner > 0)
          pup.push_back(prob(col, np, col, np, at(col, 0, TB, np, es), np, rest, inner, TB, G_BT | G_PRIO, -1.0, 1.0));
      }
      if (k == p0 + pw - 1) {
        // last block of the panel: update the trailing matrix by the panel,
        // first the next panel's columns (all rows below them, as a full
        // rectangle: what lands above the diagonal there is never read),
        // then the rest (lower tiles)
        const int64_t t0 = (int64_t)(p0 + pw) * TB;
        const int rest2 = (int)(np - t0);
        if (rest2 > 0) {
          const void* pn = at(F->L, t0, (int64_t)p0 * TB, np, es);  // trailing rows, panel columns
          const int nw = std::min(PANEL, F->nblk - (p0 + pw)) * TB;   // next panel's width
          nx.push_back(prob(pn, np, pn, np, at(F->L, t0, t0, np, es), np, rest2, nw, pw * TB, G_BT | G_PRIO, -1.0, 1.0));
          const int rest3 = rest2 - nw;
          if (rest3 > 0) {
            const void* pr = at(F->L, t0 + nw, (int64_t)p0 * TB, np, es);
            rs.push_back(prob(pr, np, pr, np, at(F->L, t0 + nw, t0 + nw, np, es), np, rest3, rest3, pw * TB,
                              G_BT | G_C_LOWER_TILES, -1.0, 1.0));
          }
        }
      }
    }
    P.job_count[k] = (int)P.jobs.size() - P.job_first[k];
    P.panel[k] = add_launch(P.sched, pan, tu.small_below[TC_PANEL]);
    P.pupd[k] = add_launch(P.sched, pup, tu.small_below[TC_PUPD]);
    P.next[k] = add_launch(P.sched, nx, tu.small_below[TC_TRAIL]);
    P.rest[k] = add_launch(P.sched, rs, tu.small_below[TC_TRAIL]);
  }
}

// Triangular inverse X = L^-1, bottom-up over a binary tree of the TB blocks:
// for the node [[A, 0], [L21, C]], T = L21 X_A then X21 = -X_C T. Leaves are
// the diagonal-block inverses. Level e of every factor runs in one launch.
//
// A single factor's plan can split (split = true) into phases by the columns
// of L they read. The split path is the root and its trailing children, up to
// SPLIT_DEPTH nodes P_0, P_1, ...; phase k holds the leading half of P_k's
// subtree and P_k's first product (columns left of P_k.mid), the last phase
// the rest: the trailing half of the deepest path node and every path node's
// second product, deepest first. Phase k can thus start as soon as the
// factorisation has finished the columns left of P_k.mid.
//
// T layout: the path nodes' T first (each survives from its first product to
// its second), then the other nodes, one level at a time (the nodes of a level
// side by side). With a split the early phases run at the same time on two
// streams, so each early phase has a region of its own for its other nodes;
// the last phase, which follows them all, reuses the first. Without a split
// the root alone takes the first place.
namespace {
size_t node_elems(const Node& nd) { return (size_t)(nd.mid - nd.a) * TB * (size_t)(nd.b - nd.mid) * TB; }
constexpr int SPLIT_DEPTH = 2;

// the split path of a factor's inverse tree (levels deepest first)
std::vector<Node> split_path(const std::vector<std::vector<Node>>& levels) {
  std::vector<Node> path;
  if (levels.empty()) return path;
  path.push_back(levels.back()[0]);
  for (int k = 1; k < SPLIT_DEPTH && (int)levels.size() > k; ++k) {
    const Node cur = path.back();
    bool found = false;
    for (const Node& nd : levels[levels.size() - 1 - k])
      if (nd.a == cur.mid && nd.b == cur.b) {
        path.push_back(nd);
        found = true;
        break;
      }
    if (!found) break;
  }
  return path;
}

bool on_path(const Node& nd, const std::vector<Node>& path) {
  for (const Node& p : path)
    if (p.a == nd.a && p.b == nd.b) return true;
  return false;
}

// phase of a node off the split path: the first path node whose leading half
// holds it, else the last phase
int node_phase(const Node& nd, const std::vector<Node>& path) {
  for (int k = 0; k < (int)path.size(); ++k)
    if (nd.b <= path[k].mid) return k;
  return (int)path.size();
}

// the split layout of T: base[k] = the start of phase k's region (k = 0..D);
// returns the elements it takes
size_t split_t_layout(const std::vector<std::vector<Node>>& levels, const std::vector<Node>& path,
                      std::vector<size_t>& base) {
  const int D = (int)path.size();
  size_t fixed = 0;
  for (const Node& nd : path) fixed += node_elems(nd);
  std::vector<size_t> need(D + 1, 0);  // per phase: the widest level of its other nodes
  for (const auto& lev : levels) {
    std::vector<size_t> s(D + 1, 0);
    for (const Node& nd : lev)
      if (!on_path(nd, path)) s[node_phase(nd, path)] += node_elems(nd);
    for (int k = 0; k <= D; ++k) need[k] = std::max(need[k], s[k]);
  }
  base.assign(D + 1, fixed);
  size_t end = fixed + std::max(need[0], need[D]);
  for (int k = 1; k < D; ++k) {
    base[k] = end;
    end += need[k];
  }
  return end;
}
}  // namespace

void plan_inverse(const std::vector<nu_factor*>& Fs, int kind, const Tuning& tu, Plan& P, bool split) {
  const bool f32 = kind != GK_F64;  // the split-BF16 products run on the FP32 copies
  std::vector<std::vector<std::vector<Node>>> lv(Fs.size());
  size_t nlev = 0;
  for (size_t i = 0; i < Fs.size(); ++i) {
    lv[i] = inverse_levels(Fs[i]->nblk);
    nlev = std::max(nlev, lv[i].size());
  }
  const size_t es = f32 ? sizeof(float) : sizeof(double);
  const int cls = kind == GK_F64 ? TC_INV64 : kind == GK_F32 ? TC_INV32 : TC_INVB;
  P.t1.clear();
  P.t2.clear();
  P.phases.clear();
  P.cuts.clear();
  // the products of one node: T = L21 X_A, X21 = -X_C T
  auto node_probs = [&](nu_factor* F, const Node& nd, size_t off_t, std::vector<GemmProblem>& p1,
                        std::vector<GemmProblem>& p2) {
    const int64_t np = F->np;
    const void* L = f32 ? (const void*)F->L32 : (const void*)F->L;
    void* X = f32 ? (void*)F->X32 : (void*)F->X;
    const int64_t a0 = (int64_t)nd.a * TB, m0 = (int64_t)nd.mid * TB;
    const int na = (nd.mid - nd.a) * TB, nc = (nd.b - nd.mid) * TB;
    void* Tn = at(F->T, 0, (int64_t)off_t, 0, es);
    p1.push_back(prob(at(L, m0, a0, np, es), np, at(X, a0, a0, np, es), np, Tn, na, nc, na, na, G_B_LOWER, 1.0, 0.0));
    p2.push_back(prob(at(X, m0, m0, np, es), np, Tn, na, at(X, m0, a0, np, es), np, nc, na, nc, G_A_LOWER, -1.0,
                      0.0));
  };
  if (split && Fs.size() == 1 && nlev >= 1) {
    nu_factor* F = Fs[0];
    const auto& levels = lv[0];
    const std::vector<Node> path = split_path(levels);
    const int D = (int)path.size();
    std::vector<size_t> path_off(D);
    size_t shared = 0;
    for (int k = 0; k < D; ++k) {
      path_off[k] = shared;
      shared += node_elems(path[k]);
      P.cuts.push_back(path[k].mid);
    }
    P.cuts.push_back(F->nblk);
    P.phases.assign(D + 1, {});
    std::vector<size_t> base;
    split_t_layout(levels, path, base);
    for (size_t e = 0; e < levels.size(); ++e) {
      std::vector<std::vector<GemmProblem>> p1(D + 1), p2(D + 1);
      std::vector<size_t> off_t = base;  // each phase's nodes of this level side by side in its region
      for (const Node& nd : levels[e]) {
        int pk = -1;
        for (int k = 0; k < D; ++k)
          if (nd.a == path[k].a && nd.b == path[k].b) pk = k;
        if (pk >= 0) {  // first product in phase pk, second in the last phase
          std::vector<GemmProblem> t1, t2;
          node_probs(F, nd, path_off[pk], t1, t2);
          p1[pk].insert(p1[pk].end(), t1.begin(), t1.end());
          p2[D].insert(p2[D].end(), t2.begin(), t2.end());
          continue;
        }
        const int ph = node_phase(nd, path);
        node_probs(F, nd, off_t[ph], p1[ph], p2[ph]);
        off_t[ph] += node_elems(nd);
      }
      for (int ph = 0; ph <= D; ++ph) {
        if (!p1[ph].empty()) P.phases[ph].push_back(add_launch(P.sched, p1[ph], tu.small_below[cls]));
        if (!p2[ph].empty()) P.phases[ph].push_back(add_launch(P.sched, p2[ph], tu.small_below[cls]));
      }
    }
    return;
  }
  for (size_t e = 0; e < nlev; ++e) {
    std::vector<GemmProblem> p1, p2;
    for (size_t i = 0; i < Fs.size(); ++i) {
      if (e >= lv[i].size()) continue;
      const bool is_root = e + 1 == lv[i].size();
      size_t off_t = is_root ? 0 : node_elems(lv[i].back()[0]);
      for (const Node& nd : lv[i][e]) {
        node_probs(Fs[i], nd, off_t, p1, p2);
        off_t += node_elems(nd);
      }
    }
    P.t1.push_back(add_launch(P.sched, p1, tu.small_below[cls]));
    P.t2.push_back(add_launch(P.sched, p2, tu.small_below[cls]));
  }
}

// room for either layout: the root, then the widest other level; or the split
// layout (the path's nodes, then a region per early phase)
size_t inverse_t_elems(int nblk) {
  const auto levels = inverse_levels(nblk);
  if (levels.empty()) return 1;
  size_t other = 0;
  for (size_t e = 0; e + 1 < levels.size(); ++e) {
    size_t s = 0;
    for (const Node& nd : levels[e]) s += node_elems(nd);
    other = std::max(other, s);
  }
  std::vector<size_t> base;
  return std::max(node_elems(levels.back()[0]) + other, split_t_layout(levels, split_path(levels), base));
}

// One Newton step X1 = 2 X - X (L X) on the blocks within w of the
// diagonal, FP64: P(I, J) = sum_{K=J..I} L(I, K) X(K, J) for I - J <= w, stored
// by column block (the blocks P(J..J+w, J) stacked), then
// X1(I, J) = 2 X(I, J) - sum_{K=J..I} X(I, K) P(K, J) for 1 <= I - J <= w, into
// the band buffer (which holds X(I, J) on entry).
void plan_band(const std::vector<nu_factor*>& Fs, int w, const Tuning& tu, Plan& P) {
  const size_t es = sizeof(double);
  const int64_t bs = (int64_t)TB * TB;
  std::vector<GemmProblem> pp, px;
  for (nu_factor* F : Fs) {
    const int64_t np = F->np;
    for (int I = 0; I < F->nblk; ++I)
      for (int d = 0; d <= w && d <= I; ++d) {
        const int J = I - d;
        pp.push_back(prob(at(F->L, (int64_t)I * TB, (int64_t)J * TB, np, es), np,
                          at(F->X, (int64_t)J * TB, (int64_t)J * TB, np, es), np,
                          F->bandP + ((int64_t)J * (w + 1) + d) * bs, TB, TB, TB, (d + 1) * TB, 0, 1.0, 0.0));
        if (d >= 1)
          px.push_back(prob(at(F->X, (int64_t)I * TB, (int64_t)J * TB, np, es), np,
                            F->bandP + (int64_t)J * (w + 1) * bs, TB, F->bandX + ((int64_t)I * (w + 1) + d) * bs,
                            TB, TB, TB, (d + 1) * TB, 0, -1.0, 2.0));
      }
  }
  P.bandp = add_launch(P.sched, pp, tu.small_below[TC_BAND]);
  P.bandx = add_launch(P.sched, px, tu.small_below[TC_BAND]);
}

nu_status plan_upload(nu_ctx* ctx, Plan& P) {
  nu_status st = check_hip(ctx, hipMalloc(&P.dprobs, std::max<size_t>(P.sched.size(), 1) * sizeof(GemmProblem)),
                           "alloc schedule");
  if (st == NU_OK && !P.sched.empty())
    st = check_hip(ctx, hipMemcpy(P.dprobs, P.sched.data(), P.sched.size() * sizeof(GemmProblem),
                                  hipMemcpyHostToDevice), "upload schedule");
  if (st == NU_OK)
    st = check_hip(ctx, hipMalloc(&P.djobs, std::max<size_t>(P.jobs.size(), 1) * sizeof(PotrfJob)), "alloc jobs");
  if (st == NU_OK && !P.jobs.empty())
    st = check_hip(ctx, hipMemcpy(P.djobs, P.jobs.data(), P.jobs.size() * sizeof(PotrfJob), hipMemcpyHostToDevice),
                   "upload jobs");
  if (st == NU_OK) P.built = true;
  return st;
}

void plan_release(Plan& P) {
  if (P.dprobs) (void)hipFree(P.dprobs);
  if (P.djobs) (void)hipFree(P.djobs);
  P = Plan();
}

// ---------------------------------------------------------------------------
// Factors

namespace {
constexpr size_t ARENA_ALIGN = 256;
size_t aligned(size_t b) { return (b + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN; }

// device bytes of each buffer of a factor of n samples, in carving order
// (prec != NU_FP64: with the reduced-precision buffers, band sized for prec;
// the T workspace holds at least t_min doubles)
std::vector<size_t> factor_buffer_bytes(int64_t n, int prec, size_t t_min) {
  const int64_t np = round_up(n, TB);
  const int nblk = (int)(np / TB);
  std::vector<size_t> b = {(size_t)np * np * sizeof(double), (size_t)np * np * sizeof(double),
                           std::max(inverse_t_elems(nblk), t_min) * sizeof(double),
                           (size_t)(nblk + FACTOR_SMALL_EXTRA) * sizeof(double), sizeof(NullFit)};
  if (prec != NU_FP64) {
    const size_t band = (size_t)nblk * (band_width(prec) + 1) * TB * TB * sizeof(double);
    b.insert(b.end(), {(size_t)np * np * sizeof(float), (size_t)np * np * sizeof(float), band, band});
  }
  return b;
}

nu_factor* new_factor(nu_ctx* ctx, int64_t n) {
  nu_factor* F = new (std::nothrow) nu_factor();
  if (!F) return nullptr;
  F->device = ctx->device;
  F->n = n;
  F->np = round_up(n, TB);
  F->nblk = (int)(F->np / TB);
  F->t_elems = inverse_t_elems(F->nblk);
  return F;
}
}  // namespace

size_t factor_bytes(int64_t n, int prec, size_t t_min) {
  size_t s = 0;
  for (size_t b : factor_buffer_bytes(n, prec, t_min)) s += aligned(b);
  return s;
}

nu_status factor_alloc(nu_ctx* ctx, int64_t n, bool own_plan, nu_factor** out) {
  *out = nullptr;
  nu_factor* F = new_factor(ctx, n);
  if (!F) return set_error(ctx, NU_ERR_OOM, "factor: host allocation");
  const int64_t np = F->np;
  nu_status st = ctx_malloc(ctx, (void**)&F->L, (size_t)np * np * sizeof(double), F->hold, "alloc L");
  if (st == NU_OK) st = ctx_malloc(ctx, (void**)&F->X, (size_t)np * np * sizeof(double), F->hold, "alloc X");
  if (st == NU_OK) st = ctx_malloc(ctx, (void**)&F->T, F->t_elems * sizeof(double), F->hold, "alloc T");
  if (st == NU_OK)
    st = ctx_malloc(ctx, (void**)&F->small, (size_t)(F->nblk + FACTOR_SMALL_EXTRA) * sizeof(double), F->hold,
                    "alloc small");
  if (st == NU_OK) st = ctx_malloc(ctx, (void**)&F->nullfit, sizeof(NullFit), F->hold, "alloc nullfit");
  if (st == NU_OK && own_plan) {
    std::vector<nu_factor*> one{F};
    plan_cholesky(one, ctx->tuning, F->plan64);
    plan_inverse(one, GK_F64, ctx->tuning, F->plan64);
    st = plan_upload(ctx, F->plan64);
  }
  if (st != NU_OK) {
    factor_free(F);
    return st;
  }
  *out = F;
  return NU_OK;
}

// A factor whose buffers (and, for prec != NU_FP64, its reduced-precision buffers) are
// carved from caller-owned device memory at *cursor (factor_bytes(n, prec)
// bytes, 256-byte aligned); the factor does not free them.
nu_status factor_place(nu_ctx* ctx, int64_t n, int prec, char** cursor, nu_factor** out, size_t t_min) {
  *out = nullptr;
  nu_factor* F = new_factor(ctx, n);
  if (!F) return set_error(ctx, NU_ERR_OOM, "factor: host allocation");
  F->owns_memory = false;
  const std::vector<size_t> sz = factor_buffer_bytes(n, prec, t_min);
  F->t_elems = std::max(F->t_elems, t_min);
  if (prec != NU_FP64) F->band_w = band_width(prec);
  void** slots[] = {(void**)&F->L,  (void**)&F->X,   (void**)&F->T,     (void**)&F->small, (void**)&F->nullfit,
                    (void**)&F->L32, (void**)&F->X32, (void**)&F->bandP, (void**)&F->bandX};
  for (size_t i = 0; i < sz.size(); ++i) {
    *slots[i] = *cursor;
    *cursor += aligned(sz[i]);
  }
  *out = F;
  return NU_OK;
}

// allocations of the reduced-precision inverse of precision prec (first use,
// and the band buffers again when a wider band is asked for)
nu_status alloc_mixed(nu_ctx* ctx, nu_factor* F, int prec) {
  const int w = band_width(prec);
  if (F->L32 && F->band_w >= w) return NU_OK;
  if (!F->owns_memory) return set_error(ctx, NU_ERR_ARG, "factor: placed without the reduced-precision buffers");
  const int64_t np = F->np;
  nu_status st = NU_OK;
  if (!F->L32) {
    st = ctx_malloc(ctx, (void**)&F->L32, (size_t)np * np * sizeof(float), F->hold, "alloc L32");
    if (st == NU_OK) st = ctx_malloc(ctx, (void**)&F->X32, (size_t)np * np * sizeof(float), F->hold, "alloc X32");
  }
  if (st == NU_OK && F->bandP) {
    st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "band realloc sync");
    (void)hipFree(F->bandP);
    (void)hipFree(F->bandX);
    F->hold.count->live -= F->band_bytes;
    F->hold.bytes -= F->band_bytes;
    F->band_bytes = 0;
    F->bandP = F->bandX = nullptr;
    F->band_w = 0;
  }
  const size_t band_elems = (size_t)F->nblk * (w + 1) * TB * TB;
  if (st == NU_OK) st = ctx_malloc(ctx, (void**)&F->bandP, band_elems * sizeof(double), F->hold, "alloc band");
  if (st == NU_OK) F->band_bytes += band_elems * sizeof(double);
  if (st == NU_OK) st = ctx_malloc(ctx, (void**)&F->bandX, band_elems * sizeof(double), F->hold, "alloc band");
  if (st == NU_OK) F->band_bytes += band_elems * sizeof(double);
  if (st == NU_OK) F->band_w = w;
  return st;
}

// the factor's own reduced-precision schedule for precision prec (the FP32
// level products reuse the FP64 T workspace: the same element count fits)
nu_status ensure_plan32(nu_ctx* ctx, nu_factor* F, int prec) {
  if (F->plan32.built && F->plan32_prec == prec) return NU_OK;
  nu_status st = alloc_mixed(ctx, F, prec);
  if (st != NU_OK) return st;
  if (F->plan32.built) {
    st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "plan rebuild sync");
    if (st != NU_OK) return st;
    plan_release(F->plan32);
  }
  std::vector<nu_factor*> one{F};
  plan_inverse(one, gemm_kind_of(prec), ctx->tuning, F->plan32, true);
  plan_band(one, band_width(prec), ctx->tuning, F->plan32);
  st = plan_upload(ctx, F->plan32);
  if (st == NU_OK) F->plan32_prec = prec;
  return st;
}

void factor_free(nu_factor* F) {
  if (!F) return;
  F->hold.release();
  if (hipSetDevice(F->device) != hipSuccess) {  // the runtime has shut down: host side only
    delete F;
    return;
  }
  (void)hipDeviceSynchronize();
  void* bufs[] = {F->L, F->X, F->T, F->small, F->nullfit, F->L32, F->X32, F->bandP, F->bandX};
  if (F->owns_memory)
    for (void* b : bufs)
      if (b) (void)hipFree(b);
  plan_release(F->plan64);
  plan_release(F->plan32);
  delete F;
}

// ---------------------------------------------------------------------------
// Enqueue sequences

nu_status launch_range(nu_ctx* ctx, const Plan& P, const Range& r, const char* name, int kind, hipStream_t s) {
  if (r.tiles == 0) return NU_OK;
  if (!s) s = ctx->stream;
  // timed through the launch's own dispatch (no marker packets around it)
  hipEvent_t e0, e1;
  timing_pair(ctx, name, &e0, &e1);
  const nu_status st =
      check_hip(ctx, launch_gemm(s, P.dprobs + r.first, r.count, r.tiles, kind, r.tile_m, r.tile_n, e0, e1), name);
  timing_add(ctx, name, e0, e1, r.flops);
  return st;
}

// Compute units the rest of a trailing update leaves to the step loop's own
// stream, so that a diagonal-block workgroup (most of a CU's LDS) finds a
// free CU while the update runs.
constexpr int LOOKAHEAD_FREE_CUS = 8;

nu_status ensure_factor_streams(nu_ctx* ctx) {
  if (ctx->s_rest) return NU_OK;
  int ncu = 0;
  nu_status st =
      check_hip(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device), "CU count");
  if (st != NU_OK) return st;
  if (ncu <= 2 * LOOKAHEAD_FREE_CUS) {  // too small to split: no lookahead
    ctx->lookahead = false;
    return NU_OK;
  }
  std::vector<uint32_t> mask((size_t)(ncu + 31) / 32, 0u);
  for (int c = LOOKAHEAD_FREE_CUS; c < ncu; ++c) mask[(size_t)c / 32] |= 1u << (c % 32);
  st = check_hip(ctx, hipStreamCreateWithFlags(&ctx->s_fac, hipStreamNonBlocking), "step-loop stream");
  if (st == NU_OK)
    st = check_hip(ctx, hipExtStreamCreateWithCUMask(&ctx->s_rest, (uint32_t)mask.size(), mask.data()),
                   "trailing-update stream");
  hipEvent_t* evs[] = {&ctx->ev_fork, &ctx->ev_pan,   &ctx->ev_rest,   &ctx->ev_join,
                       &ctx->ev_split, &ctx->ev_inv[0], &ctx->ev_inv[1]};
  for (hipEvent_t* e : evs)
    if (st == NU_OK) st = check_hip(ctx, hipEventCreateWithFlags(e, hipEventDisableTiming), "step-loop event");
  if (st != NU_OK) destroy_factor_streams(ctx);
  return st;
}

// CUs of one XCD of gfx950; a CU mask selects them XCD by XCD (bits
// [32 x, 32 x + 32) are XCD x).
constexpr int XCD_CUS = 32;

// The early inverse's streams: the first on the top `compute_units` CUs (0:
// three quarters of the chip, the fastest split on the TESS-sector curve),
// rounded to whole XCDs (at least one, at most all but one): an inverse spread
// over part of every XCD slows the factorisation's kernels more than one on
// XCDs of its own. Recreated when the count changes.
nu_status ensure_inverse_stream(nu_ctx* ctx, int compute_units) {
  int ncu = 0;
  nu_status st =
      check_hip(ctx, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device), "CU count");
  if (st != NU_OK) return st;
  if (ncu < 2 * XCD_CUS || ncu % XCD_CUS != 0) return NU_OK;  // no split: the inverse runs after the factorisation
  int c = compute_units > 0 ? compute_units : ncu / 4 * 3;
  c = std::max(XCD_CUS, std::min(ncu - XCD_CUS, (c + XCD_CUS / 2) / XCD_CUS * XCD_CUS));
  if (ctx->s_inv[0] && ctx->s_inv[1] && ctx->s_inv_cus == c) return NU_OK;
  for (hipStream_t& si : ctx->s_inv)
    if (si) {
      (void)hipStreamSynchronize(si);
      (void)hipStreamDestroy(si);
      si = nullptr;
    }
  ctx->s_inv_cus = 0;
  // the first stream (phase 0, whose products are the largest) on the top c
  // CUs; the second (phase 1, released late, small products) on every XCD but
  // the first, so that it also uses what the chain of the last steps leaves
  // idle there. A dispatch of one workgroup (a diagonal block) always starts
  // on the first XCD (workgroup i of a dispatch goes to XCD i mod 8, measured
  // with the XCC_ID register), which the second stream leaves to the chain.
  std::vector<uint32_t> mask0((size_t)(ncu + 31) / 32, 0u), mask1(mask0);
  for (int u = ncu - c; u < ncu; ++u) mask0[(size_t)u / 32] |= 1u << (u % 32);
  for (int u = XCD_CUS; u < ncu; ++u) mask1[(size_t)u / 32] |= 1u << (u % 32);
  for (int i = 0; i < 2 && st == NU_OK; ++i) {
    std::vector<uint32_t>& m = i == 0 ? mask0 : mask1;
    st = check_hip(ctx, hipExtStreamCreateWithCUMask(&ctx->s_inv[i], (uint32_t)m.size(), m.data()),
                   "early-inverse stream");
  }
  if (st == NU_OK) ctx->s_inv_cus = c;
  return st;
}

void destroy_factor_streams(nu_ctx* ctx) {
  if (ctx->s_fac) (void)hipStreamSynchronize(ctx->s_fac);
  if (ctx->s_rest) (void)hipStreamSynchronize(ctx->s_rest);
  for (hipStream_t si : ctx->s_inv)
    if (si) (void)hipStreamSynchronize(si);
  hipEvent_t* evs[] = {&ctx->ev_fork, &ctx->ev_pan,   &ctx->ev_rest,   &ctx->ev_join,
                       &ctx->ev_split, &ctx->ev_inv[0], &ctx->ev_inv[1]};
  for (hipEvent_t* e : evs)
    if (*e) {
      (void)hipEventDestroy(*e);
      *e = nullptr;
    }
  if (ctx->s_fac) (void)hipStreamDestroy(ctx->s_fac);
  if (ctx->s_rest) (void)hipStreamDestroy(ctx->s_rest);
  for (hipStream_t& si : ctx->s_inv) {
    if (si) (void)hipStreamDestroy(si);
    si = nullptr;
  }
  ctx->s_inv_cus = 0;
  ctx->s_fac = ctx->s_rest = nullptr;
}

nu_status run_factor(nu_ctx* ctx, const std::vector<nu_factor*>& Fs, const Plan& P,
                     const std::vector<const double*>& ts, const std::vector<const nu_sho*>& theta_dev,
                     const EarlyInverse* early) {
  nu_status st = NU_OK;
  for (size_t i = 0; st == NU_OK && i < Fs.size(); ++i) {
    nu_factor* F = Fs[i];
    F->inverse_kind = 0;
    st = check_hip(ctx, launch_fill_i64(ctx->stream, F->status_dev(), -1), "status init");
    if (st == NU_OK) {
      Timed tm(ctx, "kbuild", (double)F->n * (double)(F->n + 1) / 2.0);
      st = check_hip(ctx,
                     F->general ? launch_kbuild_terms(ctx->stream, ts[i], F->n, F->np, F->kernel_dev(), F->L)
                                : launch_kbuild(ctx->stream, ts[i], F->n, F->np, theta_dev[i], F->L),
                     "kbuild");
    }
  }
  if (st == NU_OK) st = run_factor_steps(ctx, P, early);
  for (size_t i = 0; st == NU_OK && i < Fs.size(); ++i)
    st = check_hip(ctx, launch_logdet_reduce(ctx->stream, Fs[i]->parts(), Fs[i]->nblk, Fs[i]->logdet_dev()),
                   "logdet");
  return st;
}

nu_status run_factor_steps(nu_ctx* ctx, const Plan& P, const EarlyInverse* early) {
  nu_status st = NU_OK;
  // Blocked right-looking Cholesky, two levels: within a panel of PANEL
  // blocks, diagonal block -> its column (times the diagonal block's inverse)
  // -> update of the panel's remaining columns; after the panel, one trailing
  // update of depth PANEL * TB on the whole chip.
  //
  // Lookahead: the trailing update after panel p is split into the next
  // panel's columns (on the step loop's stream sf) and the rest (on s_rest).
  // Panel p + 1 is factored on sf while the rest of update p runs, which
  // hides the latency-bound diagonal blocks behind the dense update. Ordering:
  //  * rest(p) needs panel p factored (ev_pan) and follows rest(p - 1) (same stream);
  //  * next(p) writes tiles that rest(p - 1) also writes, so sf waits for
  //    rest(p - 1) (ev_rest) before next(p), and so before panel p + 1;
  //  * everything else touches disjoint tiles (next(p) and panel p + 1 the
  //    next panel's columns, rest(p) only those right of them), and both read
  //    panel p's columns, which are final.
  //
  // Under stream capture the loop stays on the caller's stream: the
  // CU-masked stream is a blocking stream, whose launches HIP orders after
  // the null stream's pending work, and that must not enter a capture.
  // A step whose diagonal blocks outnumber the free CUs (a batch: one block
  // per curve) would queue them behind the update's tiles; it stays serial.
  //
  // Early inverse (early != nullptr, lookahead only): once step cuts[k] - 1
  // has factored its panel, the columns left of cuts[k] are final, and phase
  // k of the split reduced-precision inverse runs on s_inv[k % 2] (part of the
  // chip, see ensure_inverse_stream) beside the remaining steps, which from the
  // middle on are bound by the chain of diagonal blocks and leave most of the
  // chip idle. The phases write only the factor's FP32 copies and T, which no
  // step reads. The join waits for them; the caller then enqueues the rest.
  hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
  if (st == NU_OK) st = check_hip(ctx, hipStreamIsCapturing(ctx->stream, &capturing), "capture status");
  int max_jobs = 0;
  for (int c : P.job_count) max_jobs = std::max(max_jobs, c);
  const bool want_la = ctx->lookahead && capturing == hipStreamCaptureStatusNone && max_jobs <= LOOKAHEAD_FREE_CUS;
  if (st == NU_OK && want_la) st = ensure_factor_streams(ctx);
  const bool la = st == NU_OK && want_la && ctx->lookahead && ctx->s_rest;
  if (st == NU_OK && la && early) st = ensure_inverse_stream(ctx, ctx->prefetch_cus);
  hipStream_t sf = ctx->stream;
  if (la) {
    st = check_hip(ctx, hipEventRecord(ctx->ev_fork, ctx->stream), "fork");
    if (st == NU_OK) st = check_hip(ctx, hipStreamWaitEvent(ctx->s_fac, ctx->ev_fork, 0), "fork");
    sf = ctx->s_fac;
  }
  bool rest_pending = false, inv_pending[2] = {false, false};
  const int steps = (int)P.job_first.size();
  // the early phases of the inverse and the steps that release them
  const bool early_ok = la && early && ctx->s_inv[0] && ctx->s_inv[1] && early->F->plan32.built &&
                        early->F->plan32_prec == early->prec && early->F->plan32.phases.size() >= 2;
  const int early_phases = early_ok ? (int)early->F->plan32.phases.size() - 1 : 0;
  int next_phase = 0;
  if (early) early->started = 0;
  for (int k = 0; st == NU_OK && k < steps; ++k) {
    {
      Timed tm(ctx, sf, "potrf_diag", (double)P.job_count[k] * TB * TB * TB * 2.0 / 3.0);
      st = check_hip(ctx, launch_potrf_diag(sf, P.djobs + P.job_first[k], P.job_count[k]), "potrf_diag");
    }
    if (st == NU_OK) st = launch_range(ctx, P, P.panel[k], "gemm_f64:panel", GK_F64, sf);
    if (st == NU_OK) st = launch_range(ctx, P, P.pupd[k], "gemm_f64:panel_update", GK_F64, sf);
    while (st == NU_OK && next_phase < early_phases && k == early->F->plan32.cuts[next_phase] - 1) {
      // the phases share no buffer (each has its own T region), so phase k
      // does not wait for phase k - 1
      const int si = next_phase % 2;
      st = check_hip(ctx, hipEventRecord(ctx->ev_split, sf), "early inverse");
      if (st == NU_OK) st = check_hip(ctx, hipStreamWaitEvent(ctx->s_inv[si], ctx->ev_split, 0), "early inverse");
      if (st == NU_OK)
        st = run_inverse_phase(ctx, early->F, early->F->plan32, early->prec, next_phase, ctx->s_inv[si]);
      if (st == NU_OK) st = check_hip(ctx, hipEventRecord(ctx->ev_inv[si], ctx->s_inv[si]), "early inverse");
      if (st == NU_OK) {
        inv_pending[si] = true;
        early->started = ++next_phase;
      }
    }
    if (st != NU_OK || (P.next[k].tiles == 0 && P.rest[k].tiles == 0)) continue;
    if (!la) {
      st = launch_range(ctx, P, P.next[k], "gemm_f64:trailing", GK_F64, sf);
      if (st == NU_OK) st = launch_range(ctx, P, P.rest[k], "gemm_f64:trailing", GK_F64, sf);
      continue;
    }
    st = check_hip(ctx, hipEventRecord(ctx->ev_pan, sf), "panel event");
    if (st == NU_OK && rest_pending) st = check_hip(ctx, hipStreamWaitEvent(sf, ctx->ev_rest, 0), "rest wait");
    if (st == NU_OK) st = launch_range(ctx, P, P.next[k], "gemm_f64:trailing", GK_F64, sf);
    if (st == NU_OK && P.rest[k].tiles > 0) {
      st = check_hip(ctx, hipStreamWaitEvent(ctx->s_rest, ctx->ev_pan, 0), "panel wait");
      if (st == NU_OK) st = launch_range(ctx, P, P.rest[k], "gemm_f64:trailing", GK_F64, ctx->s_rest);
      if (st == NU_OK) st = check_hip(ctx, hipEventRecord(ctx->ev_rest, ctx->s_rest), "rest event");
      rest_pending = true;
    }
  }
  if (la) {
    // join (also after an error: the caller's stream must not run ahead of s_fac and s_rest)
    nu_status sj = NU_OK;
    if (rest_pending) sj = check_hip(ctx, hipStreamWaitEvent(sf, ctx->ev_rest, 0), "join");
    if (sj == NU_OK) sj = check_hip(ctx, hipEventRecord(ctx->ev_join, sf), "join");
    if (sj == NU_OK) sj = check_hip(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0), "join");
    for (int si = 0; si < 2; ++si)
      if (sj == NU_OK && inv_pending[si]) sj = check_hip(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_inv[si], 0), "join");
    if (st == NU_OK) st = sj;
  }
  if (early && st != NU_OK) early->started = 0;
  return st;
}

nu_status read_factor_status(nu_ctx* ctx, const std::vector<nu_factor*>& Fs, std::vector<int64_t>& status) {
  std::vector<double> host(2 * Fs.size());
  nu_status st = NU_OK;
  for (size_t i = 0; st == NU_OK && i < Fs.size(); ++i)
    st = check_hip(ctx, hipMemcpyAsync(&host[2 * i], Fs[i]->logdet_dev(), 2 * sizeof(double),
                                       hipMemcpyDeviceToHost, ctx->stream),
                   "read logdet and status");
  if (st == NU_OK) st = check_hip(ctx, hipStreamSynchronize(ctx->stream), "gp_factor sync");
  if (st != NU_OK) return st;
  status.resize(Fs.size());
  for (size_t i = 0; i < Fs.size(); ++i) {
    Fs[i]->logdet = host[2 * i];
    std::memcpy(&status[i], &host[2 * i + 1], sizeof(int64_t));
  }
  return NU_OK;
}

nu_status run_inverse_fp64(nu_ctx* ctx, const Plan& P) {
  nu_status st = NU_OK;
  for (size_t l = 0; st == NU_OK && l < P.t1.size(); ++l) {
    st = launch_range(ctx, P, P.t1[l], "gemm_f64:inverse", GK_F64);
    if (st == NU_OK) st = launch_range(ctx, P, P.t2[l], "gemm_f64:inverse", GK_F64);
  }
  return st;
}

// Phase k < last of a split inverse (see plan_inverse) on stream s: the FP32
// copies of the factor's columns [cuts[k - 1], cuts[k]) and of their diagonal
// blocks, then the phase's products. It reads only columns left of cuts[k],
// which the factorisation has finished by its step cuts[k] - 1.
nu_status run_inverse_phase(nu_ctx* ctx, nu_factor* F, const Plan& P, int prec, int k, hipStream_t s) {
  const int kind = gemm_kind_of(prec);
  const char* level_name = kind == GK_BF16X3 ? "gemm_bf16x3:inverse" : "gemm_f32:inverse";
  const int c0 = k > 0 ? P.cuts[k - 1] : 0, c1 = P.cuts[k];
  nu_status st;
  {
    Timed tm(ctx, s, "convert", 0.0);
    st = check_hip(ctx, launch_cvt_f64_f32(s, F->L, F->L32, F->np, 0, c0, c1), "convert L");
    if (st == NU_OK) st = check_hip(ctx, launch_cvt_f64_f32(s, F->X, F->X32, F->np, 1, c0, c1), "convert X diag");
  }
  for (size_t r = 0; st == NU_OK && r < P.phases[k].size(); ++r)
    st = launch_range(ctx, P, P.phases[k][r], level_name, kind, s);
  return st;
}

// The last phase of a split inverse on the context's stream (the phases
// before it enqueued already), then the FP64 copy and the band step.
nu_status run_inverse_post(nu_ctx* ctx, nu_factor* F, const Plan& P, int prec) {
  const int w = band_width(prec);
  if (F->band_w < w) return set_error(ctx, NU_ERR_ARG, "inverse: band buffers narrower than the precision needs");
  nu_status st = run_inverse_phase(ctx, F, P, prec, (int)P.phases.size() - 1, ctx->stream);
  if (st == NU_OK) {
    Timed tm(ctx, "convert", 0.0);
    st = check_hip(ctx, launch_cvt_f32_f64(ctx->stream, F->X32, F->X, F->np), "convert X");
  }
  if (st == NU_OK) st = check_hip(ctx, launch_band_copy(ctx->stream, F->X, F->np, F->bandX, w, 1), "band copy");
  if (st == NU_OK) st = launch_range(ctx, P, P.bandp, "gemm_f64:band", GK_F64);
  if (st == NU_OK) st = launch_range(ctx, P, P.bandx, "gemm_f64:band", GK_F64);
  if (st == NU_OK) st = check_hip(ctx, launch_band_copy(ctx->stream, F->X, F->np, F->bandX, w, 0), "band copy");
  return st;
}

// Reduced-precision doubling levels (FP32, or split BF16 for
// NU_BF16X3_REFINE), then one FP64 Newton step on the blocks within the
// precision's band width of the diagonal. P holds the levels and the band
// products of every factor in Fs (their reduced-precision buffers allocated
// for prec); a single factor's split plan runs its two halves in turn.
nu_status run_inverse_mixed(nu_ctx* ctx, const std::vector<nu_factor*>& Fs, const Plan& P, int prec) {
  if (!P.phases.empty() && Fs.size() == 1) {
    nu_status st = NU_OK;
    for (int k = 0; st == NU_OK && k + 1 < (int)P.phases.size(); ++k)
      st = run_inverse_phase(ctx, Fs[0], P, prec, k, ctx->stream);
    return st == NU_OK ? run_inverse_post(ctx, Fs[0], P, prec) : st;
  }
  const int kind = gemm_kind_of(prec), w = band_width(prec);
  const char* level_name = kind == GK_BF16X3 ? "gemm_bf16x3:inverse" : "gemm_f32:inverse";
  nu_status st = NU_OK;
  for (size_t i = 0; st == NU_OK && i < Fs.size(); ++i) {
    nu_factor* F = Fs[i];
    if (F->band_w < w) return set_error(ctx, NU_ERR_ARG, "inverse: band buffers narrower than the precision needs");
    Timed tm(ctx, "convert", 0.0);
    st = check_hip(ctx, launch_cvt_f64_f32(ctx->stream, F->L, F->L32, F->np, 0, 0, F->nblk), "convert L");
    if (st == NU_OK)
      st = check_hip(ctx, launch_cvt_f64_f32(ctx->stream, F->X, F->X32, F->np, 1, 0, F->nblk), "convert X diag");
  }
  for (size_t l = 0; st == NU_OK && l < P.t1.size(); ++l) {
    st = launch_range(ctx, P, P.t1[l], level_name, kind);
    if (st == NU_OK) st = launch_range(ctx, P, P.t2[l], level_name, kind);
  }
  for (size_t i = 0; st == NU_OK && i < Fs.size(); ++i) {
    nu_factor* F = Fs[i];
    {
      Timed tm(ctx, "convert", 0.0);
      st = check_hip(ctx, launch_cvt_f32_f64(ctx->stream, F->X32, F->X, F->np), "convert X");
    }
    if (st == NU_OK) st = check_hip(ctx, launch_band_copy(ctx->stream, F->X, F->np, F->bandX, w, 1), "band copy");
  }
  if (st == NU_OK) st = launch_range(ctx, P, P.bandp, "gemm_f64:band", GK_F64);
  if (st == NU_OK) st = launch_range(ctx, P, P.bandx, "gemm_f64:band", GK_F64);
  for (size_t i = 0; st == NU_OK && i < Fs.size(); ++i)
    st = check_hip(ctx, launch_band_copy(ctx->stream, Fs[i]->X, Fs[i]->np, Fs[i]->bandX, w, 0), "band copy");
  return st;
}

// ---------------------------------------------------------------------------
// Linear search of one factor (the inverse of the requested kind in place)

namespace {
// Partials of the products with X and L (measured at N = 18000): the
// transposed products take XRC rows per partial (512: 0.96 ms for the three
// passes; 1024: 1.50; 256: 1.02), the row products RCW columns (2048: 0.89 ms;
// 1024: 0.95; 512: 1.23). Both share one partial buffer of XRC chunks.
constexpr int XRC = LIN_XRC;
constexpr int RCW = LIN_RCW;
static_assert(RCW % XRC == 0, "row-product partials fit the buffer of the transposed ones");
// rows per partial of the box sums of squares (one wave each: latency bound,
// so many; 256: 0.89 ms at N = 18000, 512: 1.02, 1024: 1.31)
constexpr int QRC = LIN_QRC;
}  // namespace

size_t linear_ws_bytes(int64_t n, int n_d, int64_t n_epochs) {
  const int64_t np = round_up(n, TB);
  const size_t xchunks = (size_t)((n + XRC - 1) / XRC), qchunks = (size_t)((n + QRC - 1) / QRC);
  const size_t yz = (size_t)np * YCOLS;
  const size_t slots = ((size_t)n_epochs + 2) / 2;  // the int32 slot-count table, in doubles
  // template shapes after the slot table
  // the lattice flag after the shapes
  return (5 * yz + xchunks * yz + qchunks * (size_t)n_d * (size_t)n_epochs + slots + MAX_SHAPE + 1) *
         sizeof(double);
}

nu_status validate_linear(nu_ctx* ctx, int64_t n, const double* f, const double* A, int m1, const int64_t* lattice,
                          int64_t n_epochs, const int32_t* dur_samples_host, int n_d, nu_precision prec,
                          const void* depth, const void* var, const void* dll, const void* valid) {
  if (!f || !lattice || !dur_samples_host || !depth || !var || !dll || !valid)
    return set_error(ctx, NU_ERR_ARG, "linear_search: null argument");
  if (m1 < 0 || m1 > MAX_M1) return set_error(ctx, NU_ERR_ARG, "linear_search: m1 must be in [0, 7]");
  if (m1 > 0 && !A) return set_error(ctx, NU_ERR_ARG, "linear_search: A is NULL with m1 > 0");
  if (n < m1 + 1) return set_error(ctx, NU_ERR_ARG, "linear_search: need n >= m1 + 1");
  if (n_d < 1 || n_d > MAX_ND) return set_error(ctx, NU_ERR_ARG, "linear_search: n_d must be in [1, 16]");
  if (n_epochs < 1 || n_epochs > ((int64_t)1 << 31))
    return set_error(ctx, NU_ERR_ARG, "linear_search: n_epochs must be in [1, 2^31]");
  if (n_epochs < n) return set_error(ctx, NU_ERR_ARG, "linear_search: n_epochs must be >= n (strict lattice)");
  for (int j = 0; j < n_d; ++j)
    if (dur_samples_host[j] < 1 || dur_samples_host[j] > MAX_DUR)
      return set_error(ctx, NU_ERR_ARG, "linear_search: durations must be in [1, 1024] slots");
  if (prec != NU_FP64 && prec != NU_FP32_REFINE && prec != NU_BF16X3_REFINE)
    return set_error(ctx, NU_ERR_ARG, "linear_search: unknown precision");
  return NU_OK;
}

nu_status run_linear(nu_ctx* ctx, nu_factor* F, const double* f, const double* A, int m1, const int64_t* lattice,
                     int64_t n_epochs, const int32_t* dur_samples_host, int n_d, int prec, double* depth,
                     double* var, double* dll, uint8_t* valid, double* null_out, double* ws,
                     const double* shapes_host) {
  const int steps = refine_steps(prec);
  const int64_t n = F->n, np = F->np;
  const int xchunks = (int)((n + XRC - 1) / XRC), rchunks = (int)((n + RCW - 1) / RCW);
  const int qchunks = (int)((n + QRC - 1) / QRC);
  const size_t yz = (size_t)np * YCOLS;
  double* V = ws;
  double* Y = V + yz;
  double* R = Y + yz;
  double* Z = R + yz;
  double* Rz = Z + yz;
  double* xpart = Rz + yz;
  double* qpart = xpart + (size_t)xchunks * yz;
  int32_t* slot_count = reinterpret_cast<int32_t*>(qpart + (size_t)qchunks * n_d * n_epochs);
  double* shapes = qpart + (size_t)qchunks * n_d * n_epochs + ((size_t)n_epochs + 2) / 2;
  int* lattice_ok = reinterpret_cast<int*>(shapes + MAX_SHAPE);
  const int nv = m1 + 1;
  const double gemv_bytes = (double)n * (double)(n + 1) / 2.0 * 8.0;
  int dmax = 0;
  for (int j = 0; j < n_d; ++j) dmax = std::max(dmax, (int)dur_samples_host[j]);

  nu_status st = NU_OK;
  if (shapes_host) {
    size_t total = 0;
    for (int j = 0; j < n_d; ++j) total += (size_t)dur_samples_host[j];
    st = ctx_upload(ctx, shapes_host, total * sizeof(double), shapes);
    if (st != NU_OK) return st;
  }
  st = check_hip(ctx, launch_lattice_check(ctx->stream, lattice, n, n_epochs, lattice_ok), "lattice_check");
  if (st == NU_OK) st = check_hip(ctx, launch_pack_v(ctx->stream, A, m1, f, n, V), "pack_v");
  if (st != NU_OK) return st;
  {
    // Y = X V, refined against L when X is a reduced-precision inverse
    Timed tm(ctx, "rows_matvec", gemv_bytes * (1 + 2 * steps));
    st = check_hip(ctx, launch_rows_matvec(ctx->stream, F->X, np, n, np, V, nv, xpart, RCW, rchunks, nullptr, 1.0, Y),
                   "rows_matvec");
    for (int r = 0; r < steps && st == NU_OK; ++r) {
      st = check_hip(ctx, launch_rows_matvec(ctx->stream, F->L, np, n, np, Y, nv, xpart, RCW, rchunks, V, -1.0, R),
                     "rows_matvec");
      if (st == NU_OK)
        st = check_hip(ctx, launch_rows_matvec(ctx->stream, F->X, np, n, np, R, nv, xpart, RCW, rchunks, Y, 1.0, Y),
                       "rows_matvec");
    }
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "null_solve", 0.0);
    st = check_hip(ctx, launch_null_solve(ctx->stream, Y, n, m1, F->logdet_dev(), lattice_ok, F->nullfit, null_out),
                   "null_solve");
  }
  if (st != NU_OK) return st;
  {
    // Z = X^T [A~ | r~0], refined against L^T when X is a reduced-precision inverse
    Timed tm(ctx, "cols_matvec", gemv_bytes * (1 + 2 * steps));
    st = check_hip(ctx, launch_cols_matvec(ctx->stream, F->X, np, n, np, Y, nv, xpart, XRC, xchunks, nullptr, 1.0, Z),
                   "cols_matvec");
    for (int r = 0; r < steps && st == NU_OK; ++r) {
      st = check_hip(ctx, launch_cols_matvec(ctx->stream, F->L, np, n, np, Z, nv, xpart, XRC, xchunks, Y, -1.0, Rz),
                     "cols_matvec");
      if (st == NU_OK)
        st = check_hip(ctx, launch_cols_matvec(ctx->stream, F->X, np, n, np, Rz, nv, xpart, XRC, xchunks, Z, 1.0, Z),
                       "cols_matvec");
    }
  }
  if (st != NU_OK) return st;
  // ascending durations (nested boxes) with their caller indices
  std::vector<int32_t> order(n_d);
  for (int j = 0; j < n_d; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return dur_samples_host[a] < dur_samples_host[b]; });
  std::vector<int32_t> sorted(2 * n_d);
  for (int k = 0; k < n_d; ++k) {
    sorted[k] = dur_samples_host[order[k]];
    sorted[n_d + k] = order[k];
  }
  if (shapes_host) {
    Timed tm(ctx, "q_template", 0.0);
    st = check_hip(ctx, launch_slot_count(ctx->stream, lattice, n, n_epochs, slot_count), "slot_count");
    if (st == NU_OK)
      st = check_hip(ctx, launch_q_template(ctx->stream, F->X, np, n, lattice, slot_count, n_epochs, sorted.data(),
                                            dur_samples_host, n_d, shapes, dmax, QRC, qchunks, qpart),
                     "q_template");
  } else {
    Timed tm(ctx, "q_partial", 0.0);
    st = check_hip(ctx, launch_slot_count(ctx->stream, lattice, n, n_epochs, slot_count), "slot_count");
    if (st == NU_OK)
      st = check_hip(ctx, launch_q_partial(ctx->stream, F->X, np, n, lattice, slot_count, n_epochs, sorted.data(),
                                           n_d, dmax, QRC, qchunks, qpart),
                     "q_partial");
  }
  if (st != NU_OK) return st;
  {
    Timed tm(ctx, "cell_epilogue", 0.0);
    st = check_hip(ctx, launch_cell_epilogue(ctx->stream, qpart, qchunks, lattice, slot_count, n, n_epochs,
                                             dur_samples_host, n_d, Z, m1, F->nullfit, depth, var, dll, valid,
                                             shapes_host ? shapes : nullptr),
                   "cell_epilogue");
  }
  return st;
}

// ---------------------------------------------------------------------------
// Per-curve search workspace of a batch (inside the factor's T region, which
// the inverse no longer needs once the linear search starts): the linear
// search's panels, partials and slot table, and the fold's packed grid.

size_t batch_search_ws_doubles(int64_t n, int n_d, int64_t n_epochs) {
  const int64_t np = round_up(n, TB);
  const size_t xchunks = (size_t)((n + XRC - 1) / XRC), qchunks = (size_t)((n + QRC - 1) / QRC);
  const size_t yz = (size_t)np * YCOLS;
  return 5 * yz + xchunks * yz + qchunks * (size_t)n_d * (size_t)n_epochs + ((size_t)n_epochs + 2) / 2 + 1;
}

void batch_carve_search_ws(CurveJob& J, double* ws, int n_d) {
  const int64_t n = J.n, np = J.np;
  J.xchunks = (int)((n + XRC - 1) / XRC);
  J.rchunks = (int)((n + RCW - 1) / RCW);
  J.qchunks = (int)((n + QRC - 1) / QRC);
  const size_t yz = (size_t)np * YCOLS;
  J.V = ws;
  J.Y = J.V + yz;
  J.R = J.Y + yz;
  J.Z = J.R + yz;
  J.Rz = J.Z + yz;
  J.xpart = J.Rz + yz;
  J.qpart = J.xpart + (size_t)J.xchunks * yz;
  double* slots = J.qpart + (size_t)J.qchunks * n_d * J.n_epochs;
  J.slot_count = reinterpret_cast<int32_t*>(slots);
  double* flag = slots + ((size_t)J.n_epochs + 2) / 2;
  J.lattice_ok = reinterpret_cast<int*>(flag);
  J.packed = nullptr;  // the packed fold grid lives outside the workspace
}

int64_t linear_stage_blocks(int stage, const CurveJob& J, int n_d);  // linear.hip

int64_t batch_stage_blocks(int stage, const CurveJob& J, int n_d, int band_w) {
  const int64_t nb = J.nblk;
  switch (stage) {
    case BS_INIT: return 0;  // one thread per curve
    case BS_KBUILD: {
      const int64_t T = J.np / 64;
      return T * (T + 1) / 2;
    }
    case BS_LOGDET: return 1;
    case BS_CVT_L: return nb * (nb + 1) / 2;
    case BS_CVT_XD: return nb;
    case BS_CVT_BACK: return nb * (nb - 1) / 2;
    case BS_BAND: return nb > 1 ? nb * band_w : 0;
    case BS_FOLD_PACK: return ((int64_t)n_d * (J.n_epochs + 64) + 255) / 256;
    case BS_BEST: return 1;
    default: return linear_stage_blocks(stage, J, n_d);
  }
}

// ---------------------------------------------------------------------------
// Periodic search

size_t periodic_ws_bytes(int n_d, int64_t n_epochs) { return fold_workspace_doubles(n_d, n_epochs) * sizeof(double); }

nu_status validate_periodic(nu_ctx* ctx, int n_d, int64_t n_epochs, double dt, int64_t n_p, int log_term_sign) {
  if (n_d < 1 || n_d > MAX_ND) return set_error(ctx, NU_ERR_ARG, "periodic_search: n_d must be in [1, 16]");
  // the fold addresses a row of the packed grid with 32-bit byte offsets
  if (n_epochs < 1 || n_epochs > ((int64_t)1 << 27))
    return set_error(ctx, NU_ERR_ARG, "periodic_search: n_epochs must be in [1, 2^27]");
  if (!(std::isfinite(dt) && dt > 0.0))
    return set_error(ctx, NU_ERR_ARG, "periodic_search: dt must be finite and > 0");
  if (n_p < 1 || n_p > ((int64_t)1 << 31) - 1)
    return set_error(ctx, NU_ERR_ARG, "periodic_search: n_p must be in [1, 2^31)");
  if (log_term_sign != 1 && log_term_sign != -1)
    return set_error(ctx, NU_ERR_ARG, "periodic_search: log_term_sign must be +1 or -1");
  return NU_OK;
}

nu_status run_periodic(nu_ctx* ctx, const double* depth, const double* var, const double* dll, const uint8_t* valid,
                       int n_d, int64_t n_epochs, double dt, const double* periods, int64_t n_p, int log_term_sign,
                       double* q_snr, int64_t* best_phase, int32_t* best_dur, double* best_depth, double* best_sigma,
                       double* best_lnp, int64_t* best_period_index, double* ws) {
  nu_status st;
  {
    // algorithmic flops: FOLD_FLOPS_PER_VISIT per event visit, n_d * n_epochs visits per period
    Timed tm(ctx, "fold", FOLD_FLOPS_PER_VISIT * (double)n_d * (double)n_epochs * (double)n_p);
    st = check_hip(ctx, launch_fold(ctx->stream, depth, var, dll, valid, n_d, n_epochs, dt, periods, n_p,
                                    log_term_sign, q_snr, best_phase, best_dur, best_depth, best_sigma, best_lnp, ws),
                   "fold");
  }
  if (st == NU_OK && best_period_index) {
    Timed tm(ctx, "best_period", 0.0);
    st = check_hip(ctx, launch_best_period(ctx->stream, q_snr, n_p, best_period_index), "best_period");
  }
  return st;
}

}  // namespace nu
