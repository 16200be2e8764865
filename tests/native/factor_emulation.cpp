// CPU emulation of the device numeric factorization, with bounds checks.
//
// Test infrastructure: it runs the library's host preparation with the factor
// left to the device (the sweep layout with placeholders, and the numeric
// plan), performs every step of the device factorization on the CPU in the
// kernels' order -- front set-up, bottom tasks, pulls, and per level of the
// piece tree the diagonal blocks, U rows, the products' output tiles as the
// GEMM tasks list them, the scatters, then the fills of the sweep layout --
// and checks every index against the buffer it falls in (and each front
// index against its column's length). Scratch buffers are filled with NaN
// before each level, so a read of an element no step wrote shows up in the
// result. The factor and the filled layout are then compared with the host
// factorization's: L and D in compressed columns, the L_CC and L_{U,C}
// blocks, every bottom record and overflow entry, and D^{-1/2}. Built with
// AddressSanitizer and UndefinedBehaviorSanitizer by the test that runs it.
//
// Usage: factor_emulation GRAPH_FILE (the format of sweep_addressing.cpp)
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

#include "../../paper_2606_31535_amd/csrc/host/graph_handle.h"
#include "../../paper_2606_31535_amd/csrc/host/numplan.h"
#include "../../paper_2606_31535_amd/csrc/host/plan.h"

using namespace peers;

namespace {

int64_t g_checks = 0;

#define REQUIRE(cond, ...)                                                      \
  do {                                                                          \
    ++g_checks;                                                                 \
    if (!(cond)) {                                                              \
      std::fprintf(stderr, "VIOLATION %s:%d: %s: ", __FILE__, __LINE__, #cond); \
      std::fprintf(stderr, __VA_ARGS__);                                        \
      std::fprintf(stderr, "\n");                                               \
      std::exit(1);                                                             \
    }                                                                           \
  } while (0)

struct Buf {
  std::vector<double> v;
  const char* name;
  double& operator()(int64_t i) {
    REQUIRE(i >= 0 && i < (int64_t)v.size(), "%s[%" PRId64 "] of %zu", name, i, v.size());
    return v[i];
  }
  // [i0, i1) lies in the buffer
  void range(int64_t i0, int64_t i1) {
    REQUIRE(i0 >= 0 && i1 <= (int64_t)v.size() && i0 <= i1, "%s[%" PRId64 ", %" PRId64 ") of %zu", name, i0, i1,
            v.size());
  }
};

double g_worst = 0.0;
const char* g_worst_what = "";
void close_to(double got, double want, const char* what, int64_t i) {
  const double d = std::fabs(got - want) / std::max(std::fabs(want), 1e-300);
  if (!(got == want) && !(d <= 1e-11)) {
    std::fprintf(stderr, "MISMATCH %s[%" PRId64 "]: %.17g vs host %.17g\n", what, i, got, want);
    std::exit(1);
  }
  if (got != want && d > g_worst) {
    g_worst = d;
    g_worst_what = what;
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s GRAPH_FILE\n", argv[0]);
    return 2;
  }
  FILE* fp = std::fopen(argv[1], "rb");
  if (!fp) { std::perror("open"); return 2; }
  int64_t n = 0, m = 0;
  int32_t ground = 0, has_coords = 0;
  bool ok = std::fread(&n, 8, 1, fp) == 1 && std::fread(&m, 8, 1, fp) == 1 && std::fread(&ground, 4, 1, fp) == 1 &&
            std::fread(&has_coords, 4, 1, fp) == 1;
  std::vector<int32_t> eu(m), ev(m);
  std::vector<double> w(m), coords(has_coords ? n * 3 : 0);
  ok = ok && std::fread(eu.data(), 4, m, fp) == (size_t)m && std::fread(ev.data(), 4, m, fp) == (size_t)m &&
       std::fread(w.data(), 8, m, fp) == (size_t)m;
  if (has_coords) ok = ok && std::fread(coords.data(), 8, n * 3, fp) == (size_t)(n * 3);
  std::fclose(fp);
  if (!ok) { std::fprintf(stderr, "short graph file\n"); return 2; }

  peers_graph_opts o{};
  o.coords = has_coords ? coords.data() : nullptr;
  GraphHandle G;
  Status st = build_graph(n, m, eu.data(), ev.data(), w.data(), ground, o, G);
  if (st != OK) { std::fprintf(stderr, "build_graph: %d %s\n", st, last_error()); return 3; }
  const Symbolic& S = G.sym;
  const int32_t N = S.N;
  FactorPlan Ph, P;  // with the host factor; with placeholders
  st = build_plan(S, &G.num, Ph);
  if (st == OK) st = build_plan(S, nullptr, P);
  if (st != OK) { std::fprintf(stderr, "build_plan: %d %s\n", st, last_error()); return 3; }
  NumericPlan Q;
  st = build_numeric_plan(G.ing, S, P, Q);
  if (st != OK) { std::fprintf(stderr, "build_numeric_plan: %d %s\n", st, last_error()); return 3; }
  const double nan = std::numeric_limits<double>::quiet_NaN();

  Buf Lx{Q.lx0, "Lx"}, D{std::vector<double>(N, nan), "D"}, r{Q.r0, "r"}, rfin{std::vector<double>(N, nan), "rfin"};
  Buf T{std::vector<double>(std::max<int64_t>(P.store_elems, kWin), 0.0), "store"};
  Buf lu{{}, "lu"}, lud{{}, "lud"}, Gb{{}, "G"};
  Buf lcc{P.lcc, "lcc"}, luc{P.luc, "luc"};
  auto front = [&](int32_t t) -> std::pair<int64_t, int64_t> {  // (base, length) of top column t
    REQUIRE(t >= 0 && t < P.ntop, "top index %d of %d", t, P.ntop);
    const Chain& C = P.chains[P.top_chain[t]];
    const int32_t j = P.top_node[t];
    REQUIRE(P.top_off[t] == C.store_base + (int64_t)(j - C.a) * C.ld, "top column %d's front", t);
    return {P.top_off[t], C.ld};
  };
  auto fidx = [&](int32_t t, int64_t d) -> int64_t {
    const auto f = front(t);
    REQUIRE(d >= 0 && d < f.second, "depth index %" PRId64 " of top column %d (length %" PRId64 ")", d, t, f.second);
    return f.first + d;
  };

  // fronts
  for (int32_t t = 0; t < P.ntop; ++t) {
    const int32_t j = P.top_node[t];
    for (int64_t p = S.colptr[j]; p < S.colptr[j + 1]; ++p) T(fidx(t, S.depth[S.rowidx[p]] - 1)) = Lx(p);
  }
  // bottom tasks
  for (size_t task = 0; task + 1 < Q.bt_ptr.size(); ++task) {
    for (int32_t x = Q.bt_ptr[task]; x < Q.bt_ptr[task + 1]; ++x) {
      const int32_t k = Q.bcol[x];
      REQUIRE(P.top_index[k] < 0, "bottom column %d is a top node", k);
      const int64_t p0 = S.colptr[k], p1 = S.colptr[k + 1];
      double s = 0.0;
      for (int64_t p = p0; p < p1; ++p) s -= Lx(p);
      const double rk = r(k), d = rk + s;
      D(k) = d;
      rfin(k) = rk;
      for (int64_t p = p0; p < p1; ++p) Lx(p) = Lx(p) / d;
      int64_t pb = Q.bpair_ptr[x];
      for (int64_t p = p0; p < p1; ++p) {
        const int32_t j = S.rowidx[p];
        if (P.top_index[j] >= 0) continue;
        const double lp = Lx(p);
        r(j) = std::fma(-lp, rk, r(j));
        const double sp = d * lp;
        for (int64_t q = p + 1; q < p1; ++q) {
          REQUIRE(pb + (q - p - 1) < Q.bpair_ptr[x + 1], "pair target of column %d", k);
          const int64_t tgt = Q.bpair[pb + (q - p - 1)];
          REQUIRE(tgt >= S.colptr[j] && tgt < S.colptr[j + 1] && S.rowidx[tgt] == S.rowidx[q],
                  "pair target of (%d, %d) in column %d", S.rowidx[q], j, k);
          Lx(tgt) = std::fma(-Lx(q), sp, Lx(tgt));
        }
        pb += p1 - p - 1;
      }
      REQUIRE(pb == Q.bpair_ptr[x + 1], "column %d used %" PRId64 " of its pair targets", k, pb - Q.bpair_ptr[x]);
    }
  }
  // pulls
  for (int32_t t = 0; t < P.ntop; ++t) {
    const int32_t j = P.top_node[t];
    double racc = 0.0;
    for (int32_t x = Q.tg_ptr[t]; x < Q.tg_ptr[t + 1]; ++x) {
      const int32_t k = Q.tg_k[x];
      const int64_t p = Q.tg_p[x];
      REQUIRE(p >= S.colptr[k] && p < S.colptr[k + 1] && S.rowidx[p] == j, "pull of column %d into %d", k, j);
      const double lp = Lx(p), sp = D(k) * lp;
      racc = std::fma(-lp, rfin(k), racc);
      for (int64_t q = p + 1; q < S.colptr[k + 1]; ++q) {
        const int64_t i = fidx(t, S.depth[S.rowidx[q]] - 1);
        T(i) = std::fma(-Lx(q), sp, T(i));
      }
    }
    r(j) += racc;
  }
  // pieces, level by level
  const int32_t np = (int32_t)Q.pieces.size();
  std::vector<int32_t> done(np, 0);
  int64_t gemm_tiles = 0;
  double gemm_fma = 0;
  for (int32_t step = 0; step < Q.steps; ++step) {
    lu.v.assign((size_t)std::max<int64_t>(Q.luc_elems, 1), nan);
    lud.v.assign((size_t)std::max<int64_t>(Q.luc_elems, 1), nan);
    Gb.v.assign((size_t)std::max<int64_t>(Q.g_elems, 1), nan);
    // diagonal blocks
    for (int32_t x = Q.lev_ptr[step]; x < Q.lev_ptr[step + 1]; ++x) {
      const int32_t pi = Q.lev_piece[x];
      const FacPiece& Pc = Q.pieces[pi];
      REQUIRE(!done[pi], "piece %d twice", pi);
      done[pi] = 1;
      REQUIRE(Pc.w >= 1 && Pc.w <= kFacPiece && Pc.b - Pc.a + 1 == Pc.w, "piece %d width %d", pi, Pc.w);
      for (int32_t v = Pc.a; v < Pc.b; ++v) REQUIRE(S.parent[v] == v + 1, "piece %d is not a chain", pi);
      REQUIRE(Pc.dp == S.depth[Pc.b] - 1, "piece %d depth", pi);
      // every descendant piece is done: each column's updates came first
      const int32_t pb = S.parent[Pc.b];
      if (pb >= 0) REQUIRE(P.top_index[pb] >= 0, "parent of piece %d is a bottom node", pi);
      const int32_t ta = P.top_index[Pc.a];
      REQUIRE(ta >= 0, "piece %d is not top", pi);
      const int32_t w = Pc.w, dp = Pc.dp;
      auto colp = [&](int32_t t, int64_t d) -> int64_t {
        REQUIRE(P.top_index[Pc.a + t] == ta + t, "top indices of piece %d", pi);
        REQUIRE(Pc.col_base + (int64_t)t * Pc.ld == P.top_off[ta + t], "piece %d column %d front", pi, t);
        return fidx(ta + t, d);
      };
      std::vector<double> blk(kFacPiece * kFacPiece, nan), es(kFacPiece), rs(kFacPiece);
      for (int32_t t = 0; t < w; ++t)
        for (int32_t i = t + 1; i < w; ++i) blk[t * kFacPiece + i] = T(colp(t, dp + w - 1 - i));
      for (int32_t t = 0; t < w; ++t) {
        double u = 0.0;
        for (int32_t e = 0; e < Pc.nU; ++e) u -= T(colp(t, Q.pu_depth[Pc.u_begin + e] - 1));
        es[t] = r(Pc.a + t) + u;
        rs[t] = r(Pc.a + t);
      }
      for (int32_t t = 0; t < w; ++t) {
        double s = 0.0;
        for (int32_t i = t + 1; i < w; ++i) s -= blk[t * kFacPiece + i];
        const double et = es[t], rt = rs[t], dv = et + s;
        D(Pc.a + t) = dv;
        rfin(Pc.a + t) = rt;
        for (int32_t i = t + 1; i < w; ++i) {
          const double l = blk[t * kFacPiece + i] / dv;
          T(colp(t, dp + w - 1 - i)) = l;
          es[i] = std::fma(-l, et, es[i]);
          rs[i] = std::fma(-l, rt, rs[i]);
        }
        for (int32_t i = t + 2; i < w; ++i) {
          const double li = blk[t * kFacPiece + i] / dv;
          for (int32_t t2 = t + 1; t2 < i; ++t2)
            blk[t2 * kFacPiece + i] = std::fma(-li, blk[t * kFacPiece + t2], blk[t2 * kFacPiece + i]);
        }
      }
      // U_P: the rows of column b above the piece, depth descending
      REQUIRE(Pc.nU == S.colptr[Pc.b + 1] - S.colptr[Pc.b], "piece %d |U_P|", pi);
      for (int32_t e = 0; e < Pc.nU; ++e) {
        const int32_t u = S.rowidx[S.colptr[Pc.b] + e];
        REQUIRE(Q.pu_depth[Pc.u_begin + e] == S.depth[u] && Q.pu_top[Pc.u_begin + e] == P.top_index[u],
                "piece %d row %d", pi, e);
      }
    }
    // U rows
    for (int32_t x = Q.ur_ptr[step]; x < Q.ur_ptr[step + 1]; ++x) {
      const int32_t pi = Q.ur_piece[x];
      const FacPiece& Pc = Q.pieces[pi];
      REQUIRE(Pc.level == Q.pieces[Q.lev_piece[Q.lev_ptr[step]]].level, "U-row tile of piece %d at another level", pi);
      const int32_t ta = P.top_index[Pc.a];
      REQUIRE(Pc.ldu >= Pc.nU && Pc.ldu % 64 == 0, "piece %d ldu", pi);
      lu.range(Pc.luc_off, Pc.luc_off + Pc.ldu * Pc.w);
      for (int32_t e = Q.ur_row0[x]; e < std::min(Q.ur_row0[x] + kFacRowTile, Pc.nU); ++e) {
        const int32_t du = Q.pu_depth[Pc.u_begin + e] - 1;
        const int32_t dtop = Pc.dp + Pc.w - 1;
        REQUIRE(du < Pc.dp, "row %d of piece %d inside the piece", e, pi);
        std::vector<double> xv(Pc.w);
        for (int32_t t = 0; t < Pc.w; ++t) xv[t] = T(fidx(ta + t, du));
        for (int32_t t = 0; t < Pc.w; ++t) {
          const double dv = D(Pc.a + t), l = xv[t] / dv, sl = l * dv;
          lu(Pc.luc_off + (int64_t)t * Pc.ldu + e) = l;
          lud(Pc.luc_off + (int64_t)t * Pc.ldu + e) = sl;
          T(fidx(ta + t, du)) = l;
          for (int32_t t2 = t + 1; t2 < Pc.w; ++t2) xv[t2] = std::fma(-sl, T(fidx(ta + t, dtop - t2)), xv[t2]);
        }
      }
    }
    // products, tile by tile as the tasks list them
    for (int64_t x = Q.gemm_ptr[step]; x < Q.gemm_ptr[step + 1]; ++x) {
      const GemmTask& tk = Q.tasks[x];
      REQUIRE(tk.prob >= 0 && tk.prob < (int32_t)Q.probs.size(), "task %" PRId64, x);
      const GemmProb& g = Q.probs[tk.prob];
      REQUIRE(g.a_buf == BUF_LUC && g.b_buf == BUF_BT && g.c_buf == BUF_G && g.gather == 0 && g.trans == 1,
              "problem %d buffers", tk.prob);
      REQUIRE(tk.k0 == 0 && tk.k1 == g.K && tk.row0 % 64 == 0 && tk.col0 % 32 == 0 && tk.row0 < g.M &&
                  tk.col0 < g.N, "task %" PRId64 " tile", x);
      // the kernel clamps rows and columns to M-1 and N-1
      lu.range(g.a_off, g.a_off + (int64_t)(g.K - 1) * g.lda + g.M);
      lud.range(g.b_off, g.b_off + (int64_t)(g.K - 1) * g.ldb + g.N);
      Gb.range(g.c_off, g.c_off + (int64_t)(g.N - 1) * g.ldc + g.M);
      const int32_t r1 = std::min(tk.row0 + 64, g.M), c1 = std::min(tk.col0 + 32, g.N);
      for (int32_t c = tk.col0; c < c1; ++c)
        for (int32_t rr = tk.row0; rr < r1; ++rr) {
          double acc = 0.0;
          for (int32_t k = 0; k < g.K; ++k)
            acc += lu.v[g.a_off + (int64_t)k * g.lda + rr] * lud.v[g.b_off + (int64_t)k * g.ldb + c];
          Gb.v[g.c_off + (int64_t)c * g.ldc + rr] = g.alpha * acc;
        }
      ++gemm_tiles;
      gemm_fma += (double)(r1 - tk.row0) * (c1 - tk.col0) * g.K;
    }
    // scatters
    for (int32_t di = Q.sc_ptr[step]; di < Q.sc_ptr[step + 1]; ++di) {
      const int32_t t = Q.sc_dest[di];
      double racc = 0.0;
      for (int32_t x = Q.sc_src_ptr[di]; x < Q.sc_src_ptr[di + 1]; ++x) {
        const FacPiece& Pc = Q.pieces[Q.sc_piece[x]];
        const int32_t e = Q.sc_pos[x];
        REQUIRE(e >= 0 && e < Pc.nU && Q.pu_top[Pc.u_begin + e] == t, "scatter source of %d", t);
        for (int32_t i = e + 1; i < Pc.nU; ++i) {
          const int64_t dst = fidx(t, Q.pu_depth[Pc.u_begin + i] - 1);
          T(dst) -= Gb(Pc.g_off + (int64_t)e * Pc.ldu + i);
        }
        double rsum = 0.0;
        for (int32_t k = 0; k < Pc.w; ++k) rsum = std::fma(-lu(Pc.luc_off + (int64_t)k * Pc.ldu + e), rfin(Pc.a + k), rsum);
        racc += rsum;
      }
      r(P.top_node[t]) += racc;
    }
  }
  for (int32_t x = 0; x < np; ++x) REQUIRE(done[x], "piece %d never factored", x);
  // fills of the sweep layout
  REQUIRE((int64_t)Q.top_x_ptr.size() == P.ntop + 1, "top_x_ptr");
  for (int32_t t = 0; t < P.ntop; ++t) {
    const int32_t j = P.top_node[t];
    const int64_t p0 = S.colptr[j];
    REQUIRE(Q.top_x_ptr[t + 1] - Q.top_x_ptr[t] == S.colptr[j + 1] - p0, "top column %d's entries", t);
    for (int64_t p = p0; p < S.colptr[j + 1]; ++p) {
      const double v = T(fidx(t, S.depth[S.rowidx[p]] - 1));
      Lx(p) = v;
      const int64_t src = Q.top_src[Q.top_x_ptr[t] + (p - p0)];
      if (src & kLxFromLuc) luc(src & ~kLxFromLuc) = v;
      else lcc(src) = v;
    }
  }
  std::vector<BNode> bnode = P.bnode;
  std::vector<BEnt> bent = P.bent;
  REQUIRE(P.coef_p.size() == P.coef_off.size(), "coefficient map");
  for (size_t x = 0; x < P.coef_p.size(); ++x) {
    const int64_t off = P.coef_off[x];
    char* base = (off & kCoefInBent) ? (char*)bent.data() : (char*)bnode.data();
    const int64_t bytes = (off & kCoefInBent) ? (int64_t)(bent.size() * sizeof(BEnt)) : (int64_t)(bnode.size() * sizeof(BNode));
    const int64_t o = off & ~kCoefInBent;
    REQUIRE(o >= 0 && o + 8 <= bytes && o % 8 == 0, "coefficient %zu at byte %" PRId64, x, o);
    const double v = -Lx(P.coef_p[x]);
    std::memcpy(base + o, &v, 8);
  }
  std::vector<double> isd(N), top_isd(P.ntop);
  for (int32_t i = 0; i < N; ++i) isd[i] = 1.0 / std::sqrt(D(i));
  for (int32_t t = 0; t < P.ntop; ++t) top_isd[t] = 1.0 / std::sqrt(D(P.top_node[t]));
  REQUIRE(Q.bottom_records == (int64_t)Q.bnode_node.size() && Q.bottom_records <= (int64_t)bnode.size(), "records");
  for (int64_t x = 0; x < Q.bottom_records; ++x) bnode[x].isd = 1.0 / std::sqrt(D(Q.bnode_node[x]));

  // against the host factorization and its layout
  for (int32_t i = 0; i < N; ++i) {
    REQUIRE(D.v[i] > 0.0, "pivot %d", i);
    close_to(D.v[i], G.num.D[i], "D", i);
    close_to(isd[i], Ph.isd[i], "isd", i);
  }
  for (int64_t p = 0; p < Q.nnz; ++p) close_to(Lx.v[p], G.num.Lx[p], "Lx", p);
  REQUIRE(lcc.v.size() == Ph.lcc.size() && luc.v.size() == Ph.luc.size(), "block sizes");
  for (size_t x = 0; x < lcc.v.size(); ++x) close_to(lcc.v[x], Ph.lcc[x], "L_CC", (int64_t)x);
  for (size_t x = 0; x < luc.v.size(); ++x) close_to(luc.v[x], Ph.luc[x], "L_UC", (int64_t)x);
  for (int32_t t = 0; t < P.ntop; ++t) close_to(top_isd[t], Ph.top_isd[t], "top_isd", t);
  REQUIRE(bnode.size() == Ph.bnode.size() && bent.size() == Ph.bent.size(), "record counts");
  for (size_t x = 0; x < bnode.size(); ++x) {
    const BNode &a = bnode[x], &b = Ph.bnode[x];
    close_to(a.isd, b.isd, "record isd", (int64_t)x);
    for (int k = 0; k < 3; ++k) close_to(a.lc[k], b.lc[k], "record lc", (int64_t)x);
    for (int k = 0; k < 2; ++k) close_to(a.tc[k], b.tc[k], "record tc", (int64_t)x);
    REQUIRE(a.tref[0] == b.tref[0] && a.tref[1] == b.tref[1] && a.slots == b.slots && a.depth == b.depth &&
                a.ent == b.ent && a.n_more == b.n_more, "record %zu layout", x);
  }
  for (size_t x = 0; x < bent.size(); ++x) {
    REQUIRE(bent[x].ref == Ph.bent[x].ref, "overflow entry %zu", x);
    close_to(bent[x].coef, Ph.bent[x].coef, "overflow coef", (int64_t)x);
  }
  std::printf("ok: N %d pieces %d steps %d luc %.1f MB G %.1f MB tiles %" PRId64 " gemm %.3g FMA; "
              "largest difference from the host factor %.2e (%s); checks %" PRId64 "\n",
              N, np, Q.steps, Q.luc_elems * 8e-6, Q.g_elems * 8e-6, gemm_tiles, gemm_fma, g_worst, g_worst_what,
              g_checks);
  return 0;
}
