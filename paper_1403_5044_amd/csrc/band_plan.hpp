// Host-side plan of the banded preconditioner: the order in which the block rows are
// eliminated and the grouping of the substitutions into super rows.  Plain C++ (no
// device code), shared by the preconditioner and its host-logic tests.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <vector>

namespace sw {

// Limits of one super-row step's kernel arguments (rows and operator blocks).
constexpr int kMaxSuperRows = 16;
constexpr int kMaxSuperTerms = 184;

// ---- elimination order ----------------------------------------------------------------
// The band is eliminated from both ends: the top rows [0, k) downwards and the bottom
// rows [k+q, M) upwards form two chains that share no block (a separator of q rows keeps
// them more than q apart), so their steps run side by side in the same launches.  The
// separator rows [k, k+q) go last.  Position p of the order eliminates block row ord[p];
// the factors are those of block LU of the band with rows and columns in that order.
struct Order {
    int k = 0, nB = 0;
    std::vector<int> ord, rank;  // position -> block row, block row -> position
};

inline Order make_order(int M, int q) {
    Order o;
    o.k = (M - q + 1) / 2;
    o.nB = M - q - o.k;
    for (int l = 0; l < o.k; ++l) o.ord.push_back(l);
    for (int l = M - 1; l >= o.k + q; --l) o.ord.push_back(l);
    for (int l = o.k; l < o.k + q; ++l) o.ord.push_back(l);
    o.rank.assign(M, 0);
    for (int p = 0; p < M; ++p) o.rank[o.ord[p]] = p;
    return o;
}

// Factorisation step that eliminates block row l.
inline int elim_step(const Order& o, int l) {
    const int p = o.rank[l];
    if (p < o.k) return p;
    if (p < o.k + o.nB) return p - o.k;
    return std::max(o.k, o.nB) + (p - o.k - o.nB);
}

// ---- super-row substitution -----------------------------------------------------------
// The block substitutions are regrouped into super rows: runs of b consecutive positions
// of the elimination order inside one of its three segments.  Forward (L unit lower in
// that order): the blocks y_R of a super row R satisfy
//     A_R y_R = t_R - C_R y_ext,   A_R = I + (L inside R),
// with y_ext the earlier rows that R couples to, so y_R = W_R [y_ext; t_R] with
// W_R = A_R^{-1} [-C_R | I].  Backward (x_r = Dinv_r y_r - sum G_{r,c} x_c over later c):
// x_R = W'_R [y_R; x_ext], W'_R = B_R^{-1} [Dg_R | -C'_R], B_R = I + (G inside R).  W and
// W' are formed once by block substitution on their right-hand sides (GEMMs), keeping
// only the nonzero blocks.  A top and a bottom super row depend on each other in neither
// sweep, so each pair runs as one launch.
struct SuperRow {
    std::vector<int> rows;             // block rows in elimination order
    std::vector<int> ext;              // coupled rows outside R: earlier (fwd) / later (bwd)
    std::vector<std::vector<int>> id;  // [rows][inputs]: operator block index or -1
    int terms = 0;
};
struct SuperPlan {
    int b = 0;
    std::vector<SuperRow> fwd, bwd;          // fwd[i] and bwd[i] cover the same rows
    std::vector<std::vector<int>> stages;    // super rows launched together, forward order
    size_t nblocks = 0;
};

inline bool coupled(int r, int c, int q) { return r != c && std::abs(r - c) <= q; }

// Nonzero block pattern of W (forward) or W' (backward) of the super row with rows R.
// Forward inputs are [y_ext..., t_R...]; backward [y_R..., x_ext...].
inline SuperRow make_super_row(const Order& o, int q, const std::vector<int>& R, bool fwd,
                        size_t& next) {
    SuperRow S;
    S.rows = R;
    const int nb = (int)R.size();
    const int p0 = o.rank[R.front()], p1 = o.rank[R.back()];
    const int M = (int)o.ord.size();
    for (int c = 0; c < M; ++c) {
        const int pc = o.rank[c];
        if (fwd ? pc >= p0 : pc <= p1) continue;
        for (int r : R)
            if (coupled(r, c, q)) {
                S.ext.push_back(c);
                break;
            }
    }
    const int ne = (int)S.ext.size(), nin = nb + ne;
    std::vector<std::vector<char>> nz(nb, std::vector<char>(nin, 0));
    if (fwd) {
        for (int i = 0; i < nb; ++i) {
            for (int c = 0; c < ne; ++c) nz[i][c] = coupled(R[i], S.ext[c], q);
            nz[i][ne + i] = 1;
            for (int j = 0; j < i; ++j)
                if (coupled(R[i], R[j], q))
                    for (int c = 0; c < nin; ++c) nz[i][c] |= nz[j][c];
        }
    } else {
        for (int i = nb - 1; i >= 0; --i) {
            nz[i][i] = 1;
            for (int c = 0; c < ne; ++c) nz[i][nb + c] = coupled(R[i], S.ext[c], q);
            for (int j = i + 1; j < nb; ++j)
                if (coupled(R[i], R[j], q))
                    for (int c = 0; c < nin; ++c) nz[i][c] |= nz[j][c];
        }
    }
    S.id.assign(nb, std::vector<int>(nin, -1));
    for (int i = 0; i < nb; ++i)
        for (int c = 0; c < nin; ++c)
            if (nz[i][c]) {
                S.id[i][c] = (int)next++;
                ++S.terms;
            }
    return S;
}

// Super rows of b positions per segment (fewer for the separator if its rows do not fit
// one step); b = 0 if b = 1 would be needed.
inline SuperPlan plan_super(const Order& o, int q, int b) {
    SuperPlan P;
    if (b <= 1) return P;
    P.b = b;
    const int M = (int)o.ord.size();
    size_t next = 0;
    auto add = [&](int pa, int pb) {  // positions [pa, pb)
        std::vector<int> R(o.ord.begin() + pa, o.ord.begin() + pb);
        P.fwd.push_back(make_super_row(o, q, R, true, next));
        P.bwd.push_back(make_super_row(o, q, R, false, next));
        return (int)P.fwd.size() - 1;
    };
    std::vector<int> top, bot;
    for (int p = 0; p < o.k; p += b) top.push_back(add(p, std::min(p + b, o.k)));
    for (int p = o.k; p < o.k + o.nB; p += b) bot.push_back(add(p, std::min(p + b, o.k + o.nB)));
    auto fits = [&](const std::vector<int>& st) {
        int rows = 0, tf = 0, tb = 0;
        for (int i : st) {
            rows += (int)P.fwd[i].rows.size();
            tf += P.fwd[i].terms;
            tb += P.bwd[i].terms;
        }
        return rows <= kMaxSuperRows && std::max(tf, tb) <= kMaxSuperTerms;
    };
    for (size_t j = 0; j < std::max(top.size(), bot.size()); ++j) {
        std::vector<int> st;
        if (j < top.size()) st.push_back(top[j]);
        if (j < bot.size()) st.push_back(bot[j]);
        if (st.size() == 2 && !fits(st)) {
            P.stages.push_back({st[0]});
            P.stages.push_back({st[1]});
        } else {
            P.stages.push_back(st);
        }
    }
    for (int p = o.k + o.nB; p < M;) {
        int e = std::min(p + b, M);
        const size_t mark = next;
        int i = add(p, e);
        while (!fits({i}) && e - p > 1) {  // shrink the separator's super row
            P.fwd.pop_back();
            P.bwd.pop_back();
            next = mark;
            --e;
            i = add(p, e);
        }
        P.stages.push_back({i});
        p = e;
    }
    for (const auto& st : P.stages)
        if (!fits(st)) return SuperPlan{};
    P.nblocks = next;
    return P;
}

// Super-row height: b N near `target` grid rows (N: block size), lowered until every
// step fits the kernel's argument block; 0 (one block row per step) if no b > 1 fits.
inline SuperPlan choose_super(int N, const Order& o, int q, double target) {
    const int M = (int)o.ord.size();
    if (q == 0) return SuperPlan{};
    int b = (int)std::lround(target / N);
    b = std::min({b, M, kMaxSuperRows});
    for (; b > 1; --b) {
        SuperPlan P = plan_super(o, q, b);
        if (P.b > 1) return P;
    }
    return SuperPlan{};
}

}  // namespace sw
