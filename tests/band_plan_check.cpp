// Host-logic check of the banded preconditioner's plan (band_plan.hpp) over many mesh
// shapes: the elimination order (a permutation; chains that share no coupling; no fill
// outside the band; steps consistent with the order) and the super rows (a partition of
// the order into runs inside one segment; coupling sets and operator patterns against
// brute force and a numerical substitution with random values; stages that fit the
// kernel arguments and respect the dependencies of both sweeps).  Prints "ok" and exits
// with 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "band_plan.hpp"

using namespace sw;

static int g_fail = 0;
static long g_checked = 0;

#define CHECK(cond, ...)                                                 \
    do {                                                                 \
        ++g_checked;                                                     \
        if (!(cond) && g_fail++ < 20) {                                  \
            std::printf("FAIL line %d: ", __LINE__);                     \
            std::printf(__VA_ARGS__);                                    \
            std::printf("\n");                                           \
        }                                                                \
    } while (0)

static int segment(const Order& o, int p) { return p < o.k ? 0 : (p < o.k + o.nB ? 1 : 2); }

static void check_order(int M, int q) {
    const Order o = make_order(M, q);
    CHECK((int)o.ord.size() == M && (int)o.rank.size() == M, "M=%d q=%d sizes", M, q);
    if ((int)o.ord.size() != M) return;
    std::vector<int> seen(M, 0);
    for (int r : o.ord)
        if (r >= 0 && r < M) seen[r]++;
    for (int r = 0; r < M; ++r) CHECK(seen[r] == 1, "M=%d q=%d row %d seen %d times", M, q, r, seen[r]);
    for (int p = 0; p < M; ++p) CHECK(o.rank[o.ord[p]] == p, "M=%d q=%d rank", M, q);
    CHECK(o.k + o.nB + q == M && o.k - o.nB >= 0 && o.k - o.nB <= 1, "M=%d q=%d k=%d nB=%d", M, q,
          o.k, o.nB);
    // the chains: top rows 0..k-1 in order, bottom rows M-1..k+q, never coupled to each other
    for (int p = 0; p < o.k; ++p) CHECK(o.ord[p] == p, "M=%d q=%d top order", M, q);
    for (int p = 0; p < o.nB; ++p) CHECK(o.ord[o.k + p] == M - 1 - p, "M=%d q=%d bottom order", M, q);
    for (int t = 0; t < o.k; ++t)
        for (int b = o.k + q; b < M; ++b) CHECK(b - t > q, "M=%d q=%d chains coupled", M, q);
    // symbolic block elimination in this order: every new coupling stays inside the band
    std::vector<std::vector<char>> adj(M, std::vector<char>(M, 0));
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c) adj[r][c] = std::abs(r - c) <= q;
    std::vector<char> gone(M, 0);
    for (int p = 0; p < M; ++p) {
        const int v = o.ord[p];
        gone[v] = 1;
        std::vector<int> nb;
        for (int c = 0; c < M; ++c)
            if (!gone[c] && adj[v][c]) nb.push_back(c);
        for (int i : nb)
            for (int j : nb)
                if (!adj[i][j]) {
                    CHECK(std::abs(i - j) <= q, "M=%d q=%d fill (%d,%d)", M, q, i, j);
                    adj[i][j] = 1;
                }
    }
    // steps: one or two rows each (top and bottom, uncoupled), in the order's dependencies
    const int nsteps = std::max(o.k, o.nB) + q;
    std::vector<std::vector<int>> by_step(nsteps);
    for (int r = 0; r < M; ++r) {
        const int s = elim_step(o, r);
        CHECK(s >= 0 && s < nsteps, "M=%d q=%d step %d", M, q, s);
        if (s >= 0 && s < nsteps) by_step[s].push_back(r);
    }
    for (int s = 0; s < nsteps; ++s) {
        CHECK(!by_step[s].empty() && by_step[s].size() <= 2, "M=%d q=%d step %d rows", M, q, s);
        if (by_step[s].size() == 2)
            CHECK(std::abs(by_step[s][0] - by_step[s][1]) > q, "M=%d q=%d step %d coupled", M, q, s);
    }
    for (int r = 0; r < M; ++r)
        for (int c = 0; c < M; ++c)
            if (coupled(r, c, q) && o.rank[c] < o.rank[r])
                CHECK(elim_step(o, c) < elim_step(o, r), "M=%d q=%d step order %d %d", M, q, c, r);
}

// Numerical substitution with random scalar blocks: every nonzero of W (forward) or W'
// (backward) must have an operator block in the plan.
static void check_pattern(const Order& o, int q, const SuperRow& R, bool fwd, std::mt19937& rng) {
    std::uniform_real_distribution<double> U(0.5, 1.5);
    const int nb = (int)R.rows.size(), ne = (int)R.ext.size(), nin = nb + ne;
    std::vector<std::vector<double>> X(nb, std::vector<double>(nin, 0.0));
    std::vector<std::vector<double>> T(nb, std::vector<double>(nb, 0.0));  // coupling in R
    for (int i = 0; i < nb; ++i) {
        for (int c = 0; c < ne; ++c)
            if (coupled(R.rows[i], R.ext[c], q)) X[i][fwd ? c : nb + c] = -U(rng);
        X[i][fwd ? ne + i : i] = fwd ? 1.0 : U(rng);
        for (int j = 0; j < nb; ++j)
            if (j != i && coupled(R.rows[i], R.rows[j], q) && (fwd ? j < i : j > i)) T[i][j] = U(rng);
    }
    std::vector<std::vector<double>> W = X;
    if (fwd) {
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < i; ++j)
                for (int c = 0; c < nin; ++c) W[i][c] -= T[i][j] * W[j][c];
    } else {
        for (int i = nb - 1; i >= 0; --i)
            for (int j = i + 1; j < nb; ++j)
                for (int c = 0; c < nin; ++c) W[i][c] -= T[i][j] * W[j][c];
    }
    for (int i = 0; i < nb; ++i)
        for (int c = 0; c < nin; ++c)
            if (W[i][c] != 0.0)
                CHECK(R.id[i][c] >= 0, "q=%d %s row %d input %d has no operator block", q,
                      fwd ? "fwd" : "bwd", i, c);
    (void)o;
}

static void check_plan(int M, int q, const SuperPlan& P, int bmax, std::mt19937& rng) {
    if (P.b <= 1) return;  // no plan: one block row per step
    const Order o = make_order(M, q);
    CHECK(P.b <= bmax, "M=%d q=%d b=%d > %d", M, q, P.b, bmax);
    const int ng = (int)P.fwd.size();
    CHECK(ng == (int)P.bwd.size(), "M=%d q=%d group counts", M, q);
    std::vector<int> group_of(M, -1);
    std::vector<char> is_top(ng, 0), is_bottom(ng, 0);
    for (int g = 0; g < ng; ++g) {
        const auto& rows = P.fwd[g].rows;
        CHECK(rows == P.bwd[g].rows && !rows.empty() && (int)rows.size() <= P.b,
              "M=%d q=%d group %d rows", M, q, g);
        const int p0 = o.rank[rows[0]];
        for (size_t i = 0; i < rows.size(); ++i) {
            CHECK(o.rank[rows[i]] == p0 + (int)i, "M=%d q=%d group %d not a run", M, q, g);
            CHECK(segment(o, o.rank[rows[i]]) == segment(o, p0), "M=%d q=%d group %d straddles",
                  M, q, g);
            CHECK(group_of[rows[i]] == -1, "M=%d q=%d row %d in two groups", M, q, rows[i]);
            group_of[rows[i]] = g;
        }
        is_top[g] = segment(o, p0) == 0;
        is_bottom[g] = segment(o, p0) == 1;
        const int p1 = p0 + (int)rows.size() - 1;
        for (int dir = 0; dir < 2; ++dir) {
            const SuperRow& R = dir == 0 ? P.fwd[g] : P.bwd[g];
            std::vector<int> ext;
            for (int c = 0; c < M; ++c) {
                const bool outside = dir == 0 ? o.rank[c] < p0 : o.rank[c] > p1;
                bool cpl = false;
                for (int r : rows) cpl = cpl || coupled(r, c, q);
                if (outside && cpl) ext.push_back(c);
            }
            CHECK(R.ext == ext, "M=%d q=%d group %d %s coupling set", M, q, g, dir ? "bwd" : "fwd");
            int terms = 0;
            for (const auto& row : R.id)
                for (int id : row)
                    if (id >= 0) ++terms;
            CHECK(terms == R.terms, "M=%d q=%d group %d term count", M, q, g);
            check_pattern(o, q, R, dir == 0, rng);
        }
    }
    for (int r = 0; r < M; ++r) CHECK(group_of[r] >= 0, "M=%d q=%d row %d not covered", M, q, r);
    // operator block ids: unique, dense in [0, nblocks)
    std::vector<int> used(P.nblocks, 0);
    for (int g = 0; g < ng; ++g)
        for (const SuperRow* R : {&P.fwd[g], &P.bwd[g]})
            for (const auto& row : R->id)
                for (int id : row)
                    if (id >= 0) {
                        CHECK(id < (int)P.nblocks, "M=%d q=%d id range", M, q);
                        if (id < (int)P.nblocks) used[id]++;
                    }
    for (size_t i = 0; i < used.size(); ++i) CHECK(used[i] == 1, "M=%d q=%d id %zu used %d", M, q, i, used[i]);
    // stages: every group once; one group or a top and a bottom group; within the kernel's
    // argument limits; forward inputs from earlier stages, backward inputs from later ones
    std::vector<int> stage_of(ng, -1);
    for (size_t s = 0; s < P.stages.size(); ++s) {
        const auto& st = P.stages[s];
        CHECK(st.size() == 1 || (st.size() == 2 && is_top[st[0]] && is_bottom[st[1]]),
              "M=%d q=%d stage %zu composition", M, q, s);
        int rows = 0, tf = 0, tb = 0;
        for (int g : st) {
            CHECK(stage_of[g] == -1, "M=%d q=%d group %d in two stages", M, q, g);
            stage_of[g] = (int)s;
            rows += (int)P.fwd[g].rows.size();
            tf += P.fwd[g].terms;
            tb += P.bwd[g].terms;
        }
        CHECK(rows <= kMaxSuperRows && tf <= kMaxSuperTerms && tb <= kMaxSuperTerms,
              "M=%d q=%d stage %zu too large (%d rows, %d/%d terms)", M, q, s, rows, tf, tb);
    }
    for (int g = 0; g < ng; ++g) {
        CHECK(stage_of[g] >= 0, "M=%d q=%d group %d in no stage", M, q, g);
        for (int c : P.fwd[g].ext) CHECK(stage_of[group_of[c]] < stage_of[g], "M=%d q=%d fwd dep", M, q);
        for (int c : P.bwd[g].ext) CHECK(stage_of[group_of[c]] > stage_of[g], "M=%d q=%d bwd dep", M, q);
    }
}

int main() {
    std::mt19937 rng(20260401);
    std::vector<int> Ms;
    for (int M = 2; M <= 40; ++M) Ms.push_back(M);
    for (int M : {41, 45, 61, 81, 121, 241}) Ms.push_back(M);
    long plans = 0;
    for (int M : Ms) {
        std::vector<int> qs;
        for (int q = 1; q <= std::min(M - 1, 12); ++q) qs.push_back(q);
        if (M - 1 > 12) qs.push_back(M - 1);
        for (int q : qs) {
            check_order(M, q);
            const Order o = make_order(M, q);
            for (int b : {2, 3, 4, 6, 8, 11, 16}) {
                check_plan(M, q, plan_super(o, q, b), b, rng);
                ++plans;
            }
            for (int N : {9, 31, 61, 181, 241, 361}) {
                const int bt = std::min({(int)std::lround(1000.0 / N), M, kMaxSuperRows});
                check_plan(M, q, choose_super(N, o, q, 1000.0), bt, rng);
                ++plans;
            }
        }
    }
    if (g_fail) {
        std::printf("%d of %ld checks failed\n", g_fail, g_checked);
        return 1;
    }
    std::printf("ok: %ld checks over %ld plans\n", g_checked, plans);
    return 0;
}
