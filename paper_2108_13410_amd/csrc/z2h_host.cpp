// Host runtime and C ABI of libz2h: lattice, pass planner, plans, launch
// sequences, validation and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "z2h_runtime.h"

namespace z2h {
namespace rt {

// ------------------------------------------------------------------ errors

thread_local std::string g_err;

z2h_status fail(z2h_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// ------------------------------------------------------------------ lattice

// Library numbering (see the header): h(x,y) = y*Lx + x, v(x,y) = Lx*Ly + y*Lx + x.
int link_bit(int Lx, int Ly, int x, int y, int dir) {
    x = ((x % Lx) + Lx) % Lx;
    y = ((y % Ly) + Ly) % Ly;
    return (dir ? Lx * Ly : 0) + y * Lx + x;
}

void build_masks(int Lx, int Ly, uint64_t *st, uint64_t *pl) {
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            st[y * Lx + x] = (1ull << link_bit(Lx, Ly, x, y, 0)) | (1ull << link_bit(Lx, Ly, x - 1, y, 0)) |
                             (1ull << link_bit(Lx, Ly, x, y, 1)) | (1ull << link_bit(Lx, Ly, x, y - 1, 1));
            pl[y * Lx + x] = (1ull << link_bit(Lx, Ly, x, y, 0)) | (1ull << link_bit(Lx, Ly, x, y + 1, 0)) |
                             (1ull << link_bit(Lx, Ly, x, y, 1)) | (1ull << link_bit(Lx, Ly, x + 1, y, 1));
        }
}

z2h_status check_lattice(int Lx, int Ly) {
    if (Lx < 2 || Ly < 2) return fail(Z2H_ERR_INVALID, "lattice %dx%d: Lx and Ly must be >= 2", Lx, Ly);
    if (2 * Lx * Ly > kMaxN)
        return fail(Z2H_ERR_UNSUPPORTED, "lattice %dx%d has %d links; at most %d are supported", Lx, Ly,
                    2 * Lx * Ly, kMaxN);
    return Z2H_OK;
}

LatticeDev make_latdev(int Lx, int Ly) {
    LatticeDev L;
    memset(&L, 0, sizeof L);
    const int n = 2 * Lx * Ly, ns = Lx * Ly;
    uint64_t st[kMaxStab], pl[kMaxStab];
    build_masks(Lx, Ly, st, pl);
    L.n = n;
    L.nst = ns;
    for (int k = 0; k < ns; ++k) {
        L.zmask[k] = (uint32_t)pl[k];
        L.xmask[k] = (uint32_t)st[k];
        for (int l = 0; l < n; ++l) {
            if (pl[k] >> l & 1) L.zsyn[l] |= 1u << k;
            if (st[k] >> l & 1) L.xsyn[l] |= 1u << k;
        }
    }
    return L;
}

// ------------------------------------------------------------------ planner


// Register-layout sequence covering local transform bits [x0, x1) with
// windows of g.R bits from the top; g.full = number of layouts when every
// window is complete and a straight-line kernel exists for it.
static void plan_layouts(GroupGeom &g, bool resident) {
    const int R = g.R;
    const int width = g.x1 - g.x0;
    const int need = width <= R ? 1 : 1 + (width - R + R - 1) / R;
    g.full = 0;
    if (need > kMaxLay || width < R) {
        g.nlay = kMaxLay + 1;  // rejected by check_block; nothing written
        return;
    }
    int p = g.x1 - R, prev = g.x1;
    g.nlay = 0;
    while (true) {
        if (p < g.x0) p = g.x0;
        g.p[g.nlay] = p;
        g.blo[g.nlay] = 0;
        g.bhi[g.nlay] = prev - p;
        g.nlay++;
        if (p == g.x0) break;
        prev = p;
        p -= R;
    }
    if (width % R == 0 && (resident ? full_resident_ok(R, width / R) : full_level_ok(R, width / R)))
        g.full = width / R;
}

// A layout window [p, p + R) that holds bits of both runs of a split group.
bool geom_straddles(const GroupGeom &g) {
    if (!g.hi) return false;
    const int xb = g.m - g.hi;
    for (int l = 0; l < g.nlay; ++l)
        if (g.p[l] < xb && g.p[l] + g.R > xb) return true;
    return false;
}

static int pick_R(bool c128, int m) {
    int R = c128 ? 4 : 5;
    while (R > 2 && m - R < 6) --R;  // keep at least one wave per workgroup
    return R;
}

// LDS block length of a full-window group (the kernels place local index e
// at slot(t) + u * blk, t the transformed bits, u the others).  Within a
// layout every element's address is the thread's base plus a constant, so
// bank conflicts depend on the bases only: choose the shortest block, from
// the padded span up, for which each group of lanes that fills the banks
// once (256 bytes) hits distinct banks in every layout of the first wave, or
// failing that the one with the fewest collisions.
static void choose_lds_blk(const Plan &P, GroupGeom &g) {
    g.lds_blk = 0;
    if (!g.full) return;
    const int R = g.R, G = R * g.full, x0 = g.x0, x1 = g.x1;
    // slots per 256 bytes: elements of 8 or 16 bytes, or components of 4 or
    // 8 bytes with the component exchange
    const int lb = (P.c128 ? 4 : 5) + (g.cx ? 1 : 0);
    const uint32_t nb = 1u << lb, span = (1u << G) + (1u << (G - R));
    const uint32_t lanes = std::min<uint32_t>(64, 1u << (g.m - R));
    int best_bad = 1 << 30;
    uint32_t best = span;
    for (uint32_t sft = 0; sft < nb; ++sft) {
        const uint32_t blk = span + sft;
        int bad = 0;
        for (int j = 0; j < g.full; ++j) {
            const int p = x1 - R * (j + 1);
            for (uint32_t w0 = 0; w0 < lanes; w0 += nb) {
                uint32_t hit[64] = {0};
                for (uint32_t l = w0; l < std::min(lanes, w0 + nb); ++l) {
                    const uint32_t e = ((l >> p) << (p + R)) | (l & ((1u << p) - 1u));
                    const uint32_t tb = (e >> x0) & ((1u << G) - 1u);
                    const uint32_t u = (e & ((1u << x0) - 1u)) | ((e >> x1) << x0);
                    const uint32_t a = tb + (tb >> R) + u * blk;
                    bad += hit[a & (nb - 1u)]++ ? 1 : 0;
                }
            }
        }
        if (bad < best_bad) {
            best_bad = bad;
            best = blk;
            if (!bad) break;
        }
    }
    g.lds_blk = (int32_t)best;
}

// Every group's workgroup must fit the kernels' launch bounds (64..512
// threads) and the 160 KiB of LDS of a gfx950 workgroup.
static z2h_status check_block(Plan &P) {
    for (int j = 0; j < P.K; ++j) choose_lds_blk(P, P.geom[j]);
    for (int j = 0; j < P.K; ++j) {
        const int tb = P.geom[j].m - P.geom[j].R;
        if (tb < 6 || tb > 9)
            return fail(Z2H_ERR_UNSUPPORTED, "group %d: 2^%d threads per workgroup outside [64, 512]", j, tb);
        if (P.geom[j].nlay > kMaxLay)
            return fail(Z2H_ERR_UNSUPPORTED, "group %d needs more than %d register layouts", j, kMaxLay);
        if (lds_bytes(P, P.geom[j], P.geom[j].R) > (size_t)kMaxLdsBytes)
            return fail(Z2H_ERR_UNSUPPORTED, "group %d needs %zu bytes of LDS", j,
                        lds_bytes(P, P.geom[j], P.geom[j].R));
        // the observables (and the Hamiltonian passes) transform every group
        // with whole elements in LDS, also where the Trotter passes exchange
        // one component at a time
        if (obs_lds_bytes(P, P.geom[j], P.geom[j].R) > (size_t)kMaxLdsBytes)
            return fail(Z2H_ERR_UNSUPPORTED, "group %d: the observables need %zu bytes of LDS", j,
                        obs_lds_bytes(P, P.geom[j], P.geom[j].R));
        if (P.K == 1 && !P.geom[0].full)
            return fail(Z2H_ERR_UNSUPPORTED, "no one-workgroup kernel for n = %d", P.n);
    }
    return Z2H_OK;
}

// Uniform-window planner (every group uses the same R; windows may be
// partial and then run the general pass kernel).  Used for explicit tuning
// and as the fallback when no full-window split exists.
static z2h_status plan_uniform(Plan &P, int m_pref, int m_hi, int c_min, int force_R, int force_g0) {
    const int n = P.n;
    const bool c128 = P.c128;
    memset(P.geom, 0, sizeof P.geom);
    if (n <= m_hi) {
        P.K = 1;
        GroupGeom &g = P.geom[0];
        g.m = n;
        g.x1 = n;
        g.R = force_R ? force_R : pick_R(c128, n);
        plan_layouts(g, true);
        return check_block(P);
    }
    int K = 0, m = 0;
    for (int k = 2; k <= kMaxGroups && !K; ++k)
        for (int mm = m_pref; mm <= m_hi; ++mm)
            if (mm + (k - 1) * (mm - c_min) >= n) {
                K = k;
                m = mm;
                break;
            }
    if (!K) return fail(Z2H_ERR_UNSUPPORTED, "no pass schedule for n = %d with tiles of 2^%d", n, m_hi);
    P.K = K;
    const int R = force_R ? force_R : pick_R(c128, m);
    int gbits[kMaxGroups];
    int rest = n;
    for (int j = 0; j < K; ++j) {
        const int cap = j == 0 ? m : m - c_min;
        const int share = (rest + (K - j) - 1) / (K - j);
        gbits[j] = std::min(cap, share);
        if (j == 0 && force_g0) gbits[j] = std::min(cap, force_g0);
        rest -= gbits[j];
    }
    for (int j = 0; j < K && rest > 0; ++j) {  // remainder to groups with spare capacity
        const int cap = j == 0 ? m : m - c_min;
        const int add = std::min(cap - gbits[j], rest);
        gbits[j] += add;
        rest -= add;
    }
    int b = 0;
    for (int j = 0; j < K; ++j) {
        GroupGeom &g = P.geom[j];
        g.R = R;
        if (gbits[j] < R) return fail(Z2H_ERR_UNSUPPORTED, "group of %d bits below R = %d", gbits[j], R);
        if (j == 0) {
            g.m = std::max(gbits[0], std::min(m_pref, n));
            g.x1 = gbits[0];
        } else {
            const int c = std::min(b, std::max(c_min, m_pref - gbits[j]));
            if (c + gbits[j] > m_hi) return fail(Z2H_ERR_UNSUPPORTED, "group %d does not fit a tile", j);
            g.c = c;
            g.b0 = b;
            g.m = c + gbits[j];
            g.x0 = c;
            g.x1 = c + gbits[j];
        }
        g.tiles_log2 = n - g.m;
        plan_layouts(g, false);
        b += gbits[j];
    }
    return check_block(P);
}

// Full-window planner: split the n bits into K groups whose widths are
// exact multiples NL * R of a register window with a compiled straight-line
// kernel, choosing per group the window R and the tile (carried low bits c
// for 128-byte or longer contiguous runs).  Cost: passes per step, then LDS
// layout changes per step, then complex128 windows of 32 registers.
struct GroupChoice {
    int G, R, NL, m, c;
    int np;  // tiles per block: 1, or 2 (two-tile blocks of a strided group)
    int cx = 0;  // one-tile blocks: 1 = layout changes exchange one component at a time
    int hi = 0;    // > 0: the group's top hi bits form a second run of qubits
    int at = -1;   // first qubit of the (low) run, or -1: the lowest free qubit
    int hat = -1;  // first qubit of the high run, or -1: the highest free qubits
};

static bool fit_group(const Plan &P, int j, int b0, int G, int R, int NL, int m_pref, int m_hi, int c_min,
                      GroupChoice &out) {
    const int n = P.n;
    out = {G, R, NL, 0, 0, 1};
    auto lds_ok = [&](int m) {
        GroupGeom g{};
        g.m = m;
        g.R = R;
        g.full = NL;
        g.c = j == 0 ? 0 : m - G;
        return lds_bytes(P, g, R) <= (size_t)kMaxLdsBytes;
    };
    if (j == 0) {
        // largest tile up to the preferred size that suits the window
        for (int m = std::min(std::min(m_pref, m_hi), n); m >= G; --m) {
            if (m - R < 6 || m - R > 9 || !lds_ok(m)) continue;
            out.m = m;
            out.c = 0;
            return true;
        }
        return false;
    }
    // most carried bits up to the preferred tile, at least c_min of them
    const int cmax = std::min(b0, std::max(c_min, m_pref - G));
    const int cmin = std::min(b0, c_min);
    for (int c = cmax; c >= cmin; --c) {
        const int m = c + G;
        if (m - R < 6 || m - R > 9 || m > m_hi || !lds_ok(m)) continue;
        out.m = m;
        out.c = c;
        return true;
    }
    return false;
}

static int plan_cost(const Plan &P, const GroupChoice *ch, int K) {
    int exch = 0, penalty = 0;
    for (int j = 0; j < K; ++j) {
        if (j == 0 || j == K - 1) exch += 2 * (ch[j].NL - 1);
        else exch += 2 * ch[j].NL;
        if (P.c128 && ch[j].R == 5) return 1 << 29;  // 32 double-complex registers spill
        if (!P.c128 && ch[j].R < 4) penalty += 5;
    }
    return 1000 * 2 * (K - 1) + 10 * exch + penalty;
}

struct SplitCand {
    int cost, K;
    GroupChoice g[kMaxGroups];
};

static bool search_full(const Plan &P, int K, int j, int b0, int m_pref, int m_hi, int c_min, GroupChoice *cur,
                        GroupChoice *best, int &best_cost, std::vector<SplitCand> *all = nullptr) {
    const int n = P.n;
    if (j == K) {
        if (b0 != n) return false;
        const int cost = plan_cost(P, cur, K);
        if (all && cost < (1 << 29)) {
            SplitCand sc;
            sc.cost = cost;
            sc.K = K;
            for (int i = 0; i < K; ++i) sc.g[i] = cur[i];
            all->push_back(sc);
        }
        if (cost < best_cost) {
            best_cost = cost;
            for (int i = 0; i < K; ++i) best[i] = cur[i];
        }
        return true;
    }
    bool any = false;
    for (int R = 5; R >= 2; --R)
        for (int NL = 1; NL <= kMaxLay; ++NL) {
            if (!full_level_ok(R, NL)) continue;
            const int G = R * NL;
            if (b0 + G > n) continue;
            if (j == K - 1 && b0 + G != n) continue;
            GroupChoice gc;
            if (!fit_group(P, j, b0, G, R, NL, m_pref, m_hi, c_min, gc)) continue;
            cur[j] = gc;
            any |= search_full(P, K, j + 1, b0 + G, m_pref, m_hi, c_min, cur, best, best_cost, all);
        }
    return any;
}

// Geometry of a given split (group widths, windows, tiles, carried bits).
static z2h_status apply_split(Plan &P, const GroupChoice *ch, int K) {
    const int n = P.n;
    memset(P.geom, 0, sizeof P.geom);
    P.K = K;
    // qubits taken so far; a group takes one run, or two (a split group: the
    // run at b0 and hi qubits at b1), given explicitly or from the free ones
    uint64_t taken = 0;
    auto is_free = [&](int lo, int len) {
        if (lo < 0 || len < 0 || lo + len > n) return false;
        for (int x = lo; x < lo + len; ++x)
            if (taken >> x & 1) return false;
        return true;
    };
    for (int j = 0; j < K; ++j) {
        GroupGeom &g = P.geom[j];
        const int G = ch[j].G;
        if (G <= 0 || ch[j].R < 2 || ch[j].R > 5 || ch[j].m < G || ch[j].m > 14)
            return fail(Z2H_ERR_INVALID, "bad split group %d", j);
        if (j == 0 && (ch[j].c != 0 || ch[j].hi || ch[j].at > 0)) return fail(Z2H_ERR_INVALID, "group 0 is qubits 0..G-1 and carries none");
        if (j > 0 && ch[j].m != ch[j].c + G) return fail(Z2H_ERR_INVALID, "bad split group %d", j);
        if (ch[j].hi < 0 || ch[j].hi >= G) return fail(Z2H_ERR_INVALID, "group %d: bad high-run width %d", j, ch[j].hi);
        int lowest = 0;
        while (lowest < n && (taken >> lowest & 1)) ++lowest;
        int b0 = ch[j].at >= 0 ? ch[j].at : lowest, hi = ch[j].hi, b1 = 0;
        if (hi) {
            int h = ch[j].hat;
            if (h < 0) {  // the highest free qubits
                h = n;
                while (h > 0 && (taken >> (h - 1) & 1)) --h;
                h -= hi;
            }
            b1 = h;
        } else if (ch[j].at < 0) {
            // the lowest G free qubits, one run or two
            int got = 0, x = lowest;
            while (got < G && x < n && !(taken >> x & 1)) { ++x; ++got; }
            if (got < G) {
                int y = x;
                while (y < n && (taken >> y & 1)) ++y;
                hi = G - got;
                b1 = y;
            }
        }
        const int ga = G - hi;
        if (!is_free(b0, ga) || (hi && (!is_free(b1, hi) || b1 < b0 + ga)))
            return fail(Z2H_ERR_INVALID, "group %d: qubits taken twice or out of range", j);
        if (j > 0 && ch[j].c > b0) return fail(Z2H_ERR_INVALID, "group %d: carried bits reach its qubits", j);
        for (int x = b0; x < b0 + ga; ++x) taken |= 1ull << x;
        for (int x = b1; x < b1 + hi; ++x) taken |= 1ull << x;
        g.R = ch[j].R;
        g.m = ch[j].m;
        g.c = ch[j].c;
        g.b0 = b0;
        g.x0 = g.c;
        g.x1 = g.c + G;
        g.tiles_log2 = n - g.m;
        plan_layouts(g, false);
        if (hi && b1 == b0 + ga) hi = 0;  // the two runs meet: one run
        if (hi) {
            // two separate runs: the general pass kernel (groups that are
            // not whole windows), the component-exchange pass kernels, the
            // observables, the adjoint and the Hamiltonian passes are
            // compiled for them, including windows across the two runs; the
            // other straight-line pass kernels are not
            g.hi = hi;
            g.b1 = b1;
            if (g.full && !ch[j].cx)
                return fail(Z2H_ERR_INVALID, "group %d: a group of whole windows in two runs needs ':1c'", j);
        }
        if ((ch[j].np != 1 && ch[j].np != 2) || (ch[j].cx && ch[j].np != 1))
            return fail(Z2H_ERR_INVALID, "group %d: bad tiles-per-block option", j);
        g.cx = 0;
        if (ch[j].cx) {
            if (!g.full || !cx_level_ok(g.R, g.full))
                return fail(Z2H_ERR_UNSUPPORTED, "group %d: no component-exchange kernel for window %d x %d", j, g.R,
                            g.full);
            g.cx = 1;
        }
        if (ch[j].np == 2) {
            // the block's two tiles differ in the lowest tile bit, which must
            // sit right above the carried bits (strided group) or right above
            // the tile (group 0: two adjacent chunks) for the pair to be
            // contiguous
            if ((j > 0 && g.b0 - g.c < 1) || g.tiles_log2 < 1)
                return fail(Z2H_ERR_INVALID, "group %d: two-tile blocks need tile bits next to the tile", j);
            if (!g.full || !pair_level_ok(P.c128, g.R, g.full))
                return fail(Z2H_ERR_UNSUPPORTED, "group %d: no two-tile kernel for window %d x %d", j, g.R, g.full);
            g.pair = 2;
        } else {
            g.pair = 1;
        }
    }
    const uint64_t all = n == 64 ? ~0ull : (1ull << n) - 1;
    if (taken != all) return fail(Z2H_ERR_INVALID, "split covers %d of %d bits", __builtin_popcountll(taken), n);
    return check_block(P);
}

static z2h_status plan_full(Plan &P, int m_pref, int m_hi, int c_min) {
    const int n = P.n;
    memset(P.geom, 0, sizeof P.geom);
    if (n <= m_hi) {
        // whole state in one workgroup
        const int prefs[2][4] = {{5, 4, 3, 2}, {4, 3, 5, 2}};
        for (int R : prefs[P.c128 ? 1 : 0]) {
            if (n % R || !full_resident_ok(R, n / R) || n - R < 6 || n - R > 9) continue;
            P.K = 1;
            GroupGeom &g = P.geom[0];
            g.m = n;
            g.x1 = n;
            g.R = R;
            plan_layouts(g, true);
            if (check_block(P) == Z2H_OK) return Z2H_OK;
        }
    }
    for (int K = 2; K <= kMaxGroups; ++K) {
        GroupChoice cur[kMaxGroups], best[kMaxGroups];
        int best_cost = 1 << 30;
        search_full(P, K, 0, 0, m_pref, m_hi, c_min, cur, best, best_cost);
        if (best_cost >= 1 << 29) continue;
        return apply_split(P, best, K);
    }
    return fail(Z2H_ERR_UNSUPPORTED, "no full-window schedule for n = %d", n);
}

static void plan_base(int Lx, int Ly, bool c128, Plan &P) {
    P.Lx = Lx;
    P.Ly = Ly;
    P.n = 2 * Lx * Ly;
    P.nst = Lx * Ly;
    P.c128 = c128;
    P.esize = c128 ? 16 : 8;
    P.lat = make_latdev(Lx, Ly);
    P.nt = 0;
    // group 0 (contiguous tiles) in XCD-major order: each XCD streams a
    // contiguous range of the state, measured faster on every lattice; the
    // strided groups keep the hardware order, which measured faster for them
    P.xcd = 1;
    P.tables = 1;
}

// A schedule configuration string: "split=G:R:m:c/G:R:m:c/..." (groups from
// the lowest qubits up; a group may end in ":2", two tiles per block in two
// register windows, or ":1c", one tile per block whose layout changes
// exchange the real and then the imaginary parts through half the LDS, and
// then in ":h<N>": the group's top N bits are the highest N qubits not yet
// taken, so that its tile rows are not all the state's largest stride apart)
// or
// "uniform,m=..,R=..,c=..,g0=.."; either may add
// ",nt=1" (streaming loads and stores in the general pass kernel) and
// ",xcd=<mask>" (XCD-major block order in the passes over group j when bit
// j of the mask is set).
static z2h_status plan_from_config(Plan &P, const char *cfg, int m_pref, int m_hi, int c_min) {
    int v;
    const char *q;
    if ((q = strstr(cfg, "nt=")) && sscanf(q, "nt=%d", &v) == 1) P.nt = v ? 1 : 0;
    if ((q = strstr(cfg, "xcd=")) && sscanf(q, "xcd=%d", &v) == 1) P.xcd = v & ((1 << kMaxGroups) - 1);
    if ((q = strstr(cfg, "tables=")) && sscanf(q, "tables=%d", &v) == 1) P.tables = v ? 1 : 0;
    if ((q = strstr(cfg, "split="))) {
        GroupChoice ch[kMaxGroups];
        int K = 0;
        q += 6;
        while (*q && K < kMaxGroups) {
            int G, R, m, c, np = 1, cx = 0, used = 0, used2 = 0;
            if (sscanf(q, "%d:%d:%d:%d%n", &G, &R, &m, &c, &used) != 4) break;
            q += used;
            if (*q == ':' && sscanf(q, ":%d%n", &np, &used2) == 1) {
                q += used2;
                if (*q == 'c') {  // ":1c": component exchange
                    ++q;
                    cx = 1;
                }
            }
            int hi = 0, at = -1, hat = -1;
            while (q[0] == ':' && (q[1] == 'h' || q[1] == 'a')) {
                if (q[1] == 'h') {  // ":h<N>[@<Q>]": the top N bits form a run (at qubit Q)
                    if (sscanf(q, ":h%d%n", &hi, &used2) != 1 || hi < 1)
                        return fail(Z2H_ERR_INVALID, "unreadable split in \"%s\"", cfg);
                    q += used2;
                    if (*q == '@') {
                        if (sscanf(q, "@%d%n", &hat, &used2) != 1) return fail(Z2H_ERR_INVALID, "unreadable split in \"%s\"", cfg);
                        q += used2;
                    }
                } else {  // ":at<Q>": the (low) run starts at qubit Q
                    if (sscanf(q, ":at%d%n", &at, &used2) != 1) return fail(Z2H_ERR_INVALID, "unreadable split in \"%s\"", cfg);
                    q += used2;
                }
            }
            ch[K++] = {G, R, G / std::max(R, 1), m, c, np, cx, hi, at, hat};
            if (*q != '/') break;
            ++q;
        }
        if (K == 0) return fail(Z2H_ERR_INVALID, "unreadable split in \"%s\"", cfg);
        return apply_split(P, ch, K);
    }
    if (strstr(cfg, "uniform")) {
        int mp = m_pref, mh = m_hi, fR = 0, fg0 = 0, cm = c_min;
        if ((q = strstr(cfg, "m=")) && sscanf(q, "m=%d", &v) == 1 && v >= 8 && v <= 14) mp = mh = v;
        if ((q = strstr(cfg, "R=")) && sscanf(q, "R=%d", &v) == 1 && v >= 2 && v <= 5) fR = v;
        if ((q = strstr(cfg, "c=")) && sscanf(q, "c=%d", &v) == 1 && v >= 0 && v <= 8) cm = v;
        if ((q = strstr(cfg, "g0=")) && sscanf(q, "g0=%d", &v) == 1 && v >= 2) fg0 = v;
        return plan_uniform(P, mp, mh, cm, fR, fg0);
    }
    return fail(Z2H_ERR_INVALID, "unknown schedule configuration \"%s\"", cfg);
}

// Schedules chosen by the autotuner, keyed by (n, precision, batch class).
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, std::string> g_tuned;
static bool g_tune_env_loaded = false;

static int batch_class(int batch) { return batch <= 1 ? 1 : (batch < 64 ? 8 : 64); }

static z2h_status tune_load_file(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return fail(Z2H_ERR_INVALID, "cannot open tuning cache %s", path);
    char line[512];
    std::lock_guard<std::mutex> lk(g_tune_mu);
    while (fgets(line, sizeof line, f)) {
        int n, c128, bc;
        char cfg[400];
        if (line[0] == '#') continue;
        if (sscanf(line, "%d %d %d %399s", &n, &c128, &bc, cfg) == 4) g_tuned[std::make_tuple(n, c128, bc)] = cfg;
    }
    fclose(f);
    return Z2H_OK;
}

static std::string tuned_config(int n, bool c128, int batch) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (!g_tune_env_loaded) {
            g_tune_env_loaded = true;
            const char *pth = getenv("Z2H_TUNE_CACHE");
            if (pth) {
                g_tune_mu.unlock();
                (void)tune_load_file(pth);
                g_tune_mu.lock();
            }
        }
        auto it = g_tuned.find(std::make_tuple(n, c128 ? 1 : 0, batch_class(batch)));
        if (it != g_tuned.end()) return it->second;
    }
    return std::string();
}

static void plan_limits(bool c128, int max_tile_bits, int &m_pref, int &m_hi, int &c_min) {
    c_min = c128 ? 3 : 4;                  // 128-byte contiguous runs
    const int m_lo = c128 ? 12 : 13;       // preferred tile (64 KiB + padding)
    m_hi = c128 ? 13 : 14;                 // largest tile that fits in LDS
    if (max_tile_bits) m_hi = max_tile_bits;
    m_pref = std::min(m_lo, m_hi);
}

z2h_status make_plan(int Lx, int Ly, bool c128, int max_tile_bits, Plan &P, int batch_hint) {
    z2h_status st = check_lattice(Lx, Ly);
    if (st) return st;
    plan_base(Lx, Ly, c128, P);
    if (max_tile_bits && (max_tile_bits < 8 || max_tile_bits > (c128 ? 13 : 14)))
        return fail(Z2H_ERR_INVALID, "max_tile_bits %d outside [8, %d]", max_tile_bits, c128 ? 13 : 14);
    int m_pref, m_hi, c_min;
    plan_limits(c128, max_tile_bits, m_pref, m_hi, c_min);
    // explicit override, then a tuned schedule, then the planner's own choice
    if (const char *tv = getenv("Z2H_TUNE")) {
        if (strstr(tv, "uniform") || strstr(tv, "split=")) return plan_from_config(P, tv, m_pref, m_hi, c_min);
    }
    if (!max_tile_bits) {
        const std::string cfg = tuned_config(P.n, c128, batch_hint);
        if (!cfg.empty()) {
            Plan T = P;
            if (plan_from_config(T, cfg.c_str(), m_pref, m_hi, c_min) == Z2H_OK) {
                P = T;
                return Z2H_OK;
            }
        }
    }
    // Straight-line full-window kernels unless they would cost extra passes
    // (HBM sweeps) per step compared with partial windows.
    Plan U = P;
    const z2h_status su = plan_uniform(U, m_pref, m_hi, c_min, 0, 0);
    st = plan_full(P, m_pref, m_hi, c_min);
    if (st == Z2H_OK && (su != Z2H_OK || P.K <= U.K)) return Z2H_OK;
    if (su == Z2H_OK) {
        P = U;
        return Z2H_OK;
    }
    return st;
}

// Tile options of one group of a split: every (m, c) whose block size is
// within the launch bounds and whose tile fits LDS, with contiguous runs of
// at least 64 bytes for groups that carry low bits; strided tiles too large
// for two workgroups per CU also with the component exchange.
struct TileOpt {
    int m, c, np;
    int cx = 0;
};

static std::vector<TileOpt> group_tiles(const Plan &P, int j, int b0, int G, int R, int m_hi) {
    std::vector<TileOpt> out;
    auto lds_ok = [&](int m) {
        GroupGeom g{};
        g.m = m;
        g.R = R;
        g.full = G % R == 0 ? G / R : 0;
        g.c = j == 0 ? 0 : m - G;
        return lds_bytes(P, g, R) <= (size_t)kMaxLdsBytes;
    };
    const int c_lo = P.c128 ? 2 : 3;
    const bool pair = (G % R == 0) && pair_level_ok(P.c128, R, G / R);
    if (j == 0) {
        for (int m = G; m <= std::min(m_hi, P.n); ++m)
            if (m - R >= 6 && m - R <= 9 && lds_ok(m)) {
                out.push_back({m, 0, 1});
                if (pair && m == G && P.n - m >= 1) out.push_back({m, 0, 2});
            }
        return out;
    }
    for (int c = c_lo; c <= b0; ++c) {
        const int m = c + G;
        if (m > m_hi) break;
        if (m - R >= 6 && m - R <= 9 && lds_ok(m)) {
            out.push_back({m, c, 1});
            if (pair && c >= 4 && b0 - c >= 1 && P.n - m >= 1) out.push_back({m, c, 2});
            GroupGeom g{};
            g.m = m;
            g.R = R;
            g.full = G % R == 0 ? G / R : 0;
            g.c = c;
            if (g.full && cx_level_ok(R, g.full) && 2 * lds_bytes(P, g, R) > (size_t)kMaxLdsBytes)
                out.push_back({m, c, 1, 1});
        }
    }
    return out;
}

// Candidate schedules for the autotuner.  Structures (group widths and
// register windows) come from the full-window planner with the fewest groups
// (and one more); for each structure every combination of per-group tile
// options is a candidate, best-ranked structures first.  Uniform-window
// schedules follow.
std::vector<std::string> tune_candidates(int Lx, int Ly, bool c128) {
    Plan P;
    plan_base(Lx, Ly, c128, P);
    int m_pref, m_hi, c_min;
    plan_limits(c128, 0, m_pref, m_hi, c_min);
    std::vector<std::string> out;
    std::vector<SplitCand> all;
    int Kbest = 0;
    for (int K = 2; K <= kMaxGroups; ++K) {
        for (int mp = std::max(10, m_pref - 1); mp <= m_hi; ++mp)
            for (int cm = c_min; cm <= c_min + 2; ++cm) {
                GroupChoice cur[kMaxGroups], best[kMaxGroups];
                int bc = 1 << 30;
                search_full(P, K, 0, 0, mp, m_hi, cm, cur, best, bc, &all);
            }
        if (!all.empty() && !Kbest) Kbest = K;
        if (Kbest && K > Kbest) break;
    }
    std::stable_sort(all.begin(), all.end(), [](const SplitCand &a, const SplitCand &b) { return a.cost < b.cost; });
    std::vector<std::string> seen_struct;
    const size_t kMaxCands = 64;
    for (const auto &sc : all) {
        std::string key;
        for (int j = 0; j < sc.K; ++j) key += std::to_string(sc.g[j].G) + ":" + std::to_string(sc.g[j].R) + "/";
        if (std::find(seen_struct.begin(), seen_struct.end(), key) != seen_struct.end()) continue;
        seen_struct.push_back(key);
        std::vector<std::vector<TileOpt>> opts(sc.K);
        int b0 = 0;
        size_t combos = 1;
        for (int j = 0; j < sc.K; ++j) {
            opts[j] = group_tiles(P, j, b0, sc.g[j].G, sc.g[j].R, m_hi);
            b0 += sc.g[j].G;
            combos *= opts[j].size();
        }
        if (combos == 0) continue;
        for (size_t idx = 0; idx < combos && out.size() < kMaxCands; ++idx) {
            std::string cfg = "split=";
            size_t r = idx;
            int xcd = 1;  // group 0, and the groups with the component exchange
            for (int j = 0; j < sc.K; ++j) {
                const auto &o = opts[j][r % opts[j].size()];
                r /= opts[j].size();
                char buf[64];
                snprintf(buf, sizeof buf, "%s%d:%d:%d:%d%s", j ? "/" : "", sc.g[j].G, sc.g[j].R, o.m, o.c,
                         o.np == 2 ? ":2" : (o.cx ? ":1c" : ""));
                cfg += buf;
                if (o.cx) xcd |= 1 << j;
            }
            if (xcd != 1) cfg += ",xcd=" + std::to_string(xcd);
            if (std::find(out.begin(), out.end(), cfg) == out.end()) out.push_back(cfg);
        }
        if (out.size() >= kMaxCands) break;
    }
    // Three-group schedules whose strided groups exchange one component at
    // a time: the middle group may also take part of its qubits high in the
    // state (":h<N>@<Q>"; the top group then takes the free qubits, in two
    // runs), so that neither strided group has all its rows at the largest
    // strides.  Variants of the best-ranked such schedule.
    std::vector<std::string> bases(out);
    if (P.n >= 26) {
        // two ten-qubit strided groups with the component exchange above a
        // contiguous group 0 (the structure search may rank only more groups)
        const int G0 = P.n - 20, c = c_min;
        for (int R0 : {4, 3, 5, 2}) {
            if (G0 % R0) continue;
            char buf[96];
            snprintf(buf, sizeof buf, "split=%d:%d:%d:0/10:5:%d:%d:1c/10:5:%d:%d:1c,xcd=7", G0, R0, G0, c + 10, c,
                     c + 10, c);
            Plan T;
            plan_base(Lx, Ly, c128, T);
            if (plan_from_config(T, buf, m_pref, m_hi, c_min) != Z2H_OK) continue;
            if (std::find(out.begin(), out.end(), std::string(buf)) == out.end()) out.push_back(buf);
            bases.insert(bases.begin(), buf);
            break;
        }
    }
    for (const std::string &base : bases) {
        if (base.compare(0, 6, "split=") != 0) continue;
        std::vector<std::string> grp;
        size_t a = 6, e;
        const size_t comma = base.find(',');
        const std::string body = base.substr(0, comma);
        while ((e = body.find('/', a)) != std::string::npos) {
            grp.push_back(body.substr(a, e - a));
            a = e + 1;
        }
        grp.push_back(body.substr(a));
        auto is_cx = [](const std::string &g) { return g.size() > 3 && g.compare(g.size() - 3, 3, ":1c") == 0; };
        if (grp.size() != 3 || !is_cx(grp[1]) || !is_cx(grp[2])) continue;
        const int G1 = atoi(grp[1].c_str());
        for (int hi = G1 / 2; hi <= G1 / 2 + 2 && hi < G1; ++hi)
            for (int d = 1; d <= 3; ++d) {
                const int q = P.n - hi - 1 - d;
                char buf[48];
                snprintf(buf, sizeof buf, ":h%d@%d", hi, q);
                const std::string cfg = "split=" + grp[0] + "/" + grp[1] + buf + "/" + grp[2] + ",xcd=7";
                Plan T;
                plan_base(Lx, Ly, c128, T);
                if (plan_from_config(T, cfg.c_str(), m_pref, m_hi, c_min) == Z2H_OK &&
                    std::find(out.begin(), out.end(), cfg) == out.end())
                    out.push_back(cfg);
            }
        break;
    }
    for (int m = m_hi - 2; m <= m_hi; ++m)
        for (int c = c_min; c <= c_min + 1; ++c) {
            char buf[96];
            snprintf(buf, sizeof buf, "uniform,m=%d,c=%d,nt=1", m, c);
            out.push_back(buf);
        }
    return out;
}

z2h_status plan_with_config(int Lx, int Ly, bool c128, const char *cfg, Plan &P) {
    z2h_status st = check_lattice(Lx, Ly);
    if (st) return st;
    plan_base(Lx, Ly, c128, P);
    int m_pref, m_hi, c_min;
    plan_limits(c128, 0, m_pref, m_hi, c_min);
    return plan_from_config(P, cfg, m_pref, m_hi, c_min);
}

void tune_store(int n, bool c128, int batch, const std::string &cfg) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(n, c128 ? 1 : 0, batch_class(batch))] = cfg;
}

z2h_status tune_load(const char *path) { return tune_load_file(path); }

int tune_batch_class(int batch) { return batch_class(batch); }

size_t lds_bytes(const Plan &P, const GroupGeom &g, int R) {
    size_t elems = ((size_t)1 << g.m) + ((size_t)1 << (g.m - R));
    if (g.full) {
        // full-window kernels: a block per value of the untransformed bits;
        // before the planner has chosen the block, count the longest one
        const int G = R * g.full;
        const size_t blk = g.lds_blk ? (size_t)g.lds_blk
                                     : ((size_t)1 << G) + ((size_t)1 << (G - R)) + (P.c128 ? 15 : 31);
        elems = std::max(elems, ((size_t)1 << (g.m - G)) * blk);
    }
    // exchange region (one element per slot, or one component with the
    // component exchange; it also holds the table's FP64 factors while the
    // table is built)
    size_t b = elems * (g.cx ? P.esize / 2 : P.esize);
    if (g.cx) b = (b + 15) & ~(size_t)15;
    b += (size_t)(P.nst + 1) * (P.n + 1) * P.esize;  // phase table
    b = (b + 15) & ~(size_t)15;
    b += 16 * sizeof(double);                        // block reduction
    return b;
}

size_t obs_lds_bytes(const Plan &P, const GroupGeom &g, int R) {
    const size_t elems = ((size_t)1 << g.m) + ((size_t)1 << (g.m - R));
    return ((elems * P.esize + 15) & ~(size_t)15) + 16 * sizeof(double);
}


static const int kObsWorkersMax = 1024;

int obs_workers(const GroupGeom &g) {
    const uint64_t tiles = 1ull << g.tiles_log2;
    return (int)std::min<uint64_t>(tiles, kObsWorkersMax);
}


// ------------------------------------------------------------------ timing

namespace {
thread_local bool t_timing_unused = false;
}  // namespace

thread_local bool t_timing = false;
thread_local std::vector<TimedLaunch> t_launches;
thread_local std::vector<hipEvent_t> t_pool;

hipEvent_t get_event() {
    if (!t_pool.empty()) {
        hipEvent_t e = t_pool.back();
        t_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// ------------------------------------------------------------------ launch sequences

z2h_status validate_state_ptr(const void *p, const char *what) {
    if (!p) return fail(Z2H_ERR_INVALID, "%s is NULL", what);
    if ((uintptr_t)p & 255) return fail(Z2H_ERR_INVALID, "%s is not 256-byte aligned", what);
    return Z2H_OK;
}

z2h_status validate_schedule(const Plan &P, const z2h_schedule *s) {
    if (!s) return fail(Z2H_ERR_INVALID, "schedule is NULL");
    if (s->steps < 0 || s->steps > (1ll << 30)) return fail(Z2H_ERR_INVALID, "steps = %lld out of range", (long long)s->steps);
    if (!std::isfinite(s->dt)) return fail(Z2H_ERR_INVALID, "dt is not finite");
    if (s->k_begin < 0 || s->k_end < s->k_begin || s->k_end > s->steps)
        return fail(Z2H_ERR_INVALID, "step range [%lld, %lld) not inside [0, %lld)", (long long)s->k_begin,
                    (long long)s->k_end, (long long)s->steps);
    if (s->sampling != 0 && s->sampling != 1) return fail(Z2H_ERR_INVALID, "sampling must be 0 or 1");
    if (s->order != 0 && s->order != 1) return fail(Z2H_ERR_INVALID, "order must be 0 or 1");
    const double *c[2] = {&s->start.JA, &s->end.JA};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 4; ++j)
            if (!std::isfinite(c[i][j])) return fail(Z2H_ERR_INVALID, "coupling not finite");
    (void)P;
    return Z2H_OK;
}

// Eq. (ini1)/(ini2): equal weight on the 2^(n - Np + 1) configurations with
// every plaquette (star) even; psi_1' is then Hadamard-transformed, whose
// 2^(-n/2) normalization (n even) is folded into the amplitude.
InitJob init_job(const Plan &P, int kind, uint64_t offset) {
    InitJob j;
    memset(&j, 0, sizeof j);
    j.offset = offset;
    j.kind = kind;
    const double even = 1.0 / std::sqrt(std::ldexp(1.0, P.n - P.nst + 1));
    if (kind == Z2H_INIT_PSI1) j.amp = even;
    if (kind == Z2H_INIT_PSI1P) j.amp = even * std::ldexp(1.0, -P.n / 2);
    if (kind == Z2H_INIT_PLUS) j.amp = std::ldexp(1.0, -P.n / 2);
    return j;
}

JobDev make_job(const z2h_schedule *s, uint64_t offset) {
    JobDev J;
    memset(&J, 0, sizeof J);
    J.offset = offset;
    J.steps = (int32_t)(s->k_end - s->k_begin);
    J.k_begin = (int32_t)s->k_begin;
    J.M = (int32_t)s->steps;
    J.sampling = s->sampling;
    J.order = s->order;
    J.renorm = s->renorm;
    J.dt = s->dt;
    const double *a = &s->start.JA, *b = &s->end.JA;
    for (int j = 0; j < 4; ++j) {
        J.c0[j] = a[j];
        J.c1[j] = b[j];
    }
    return J;
}

int pass_kind_of(const LevelOp &op) {
    if (op.kind == kPlainH) return 2;
    if (op.kind == kIdle) return 3;
    return op.basis == 0 ? 0 : 1;
}


void timed_begin(hipStream_t s, hipEvent_t &e0, hipEvent_t &e1) {
    e0 = e1 = nullptr;
    if (!t_timing) return;
    e0 = get_event();
    e1 = get_event();
    if (e0) (void)hipEventRecord(e0, s);
}

void timed_end(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int kind) {
    if (!t_timing || !e0 || !e1) return;
    (void)hipEventRecord(e1, s);
    t_launches.push_back({e0, e1, kind});
}

// Launch one level for the jobs of J (all on the lattice of plan P).
// Where the states of J start: a uniform stride lets the pass kernels issue
// their tile loads before reading the job record.
static void job_layout(const JobSet &J, LevelArgs &a) {
    a.jmode = 1;
    a.jbase = 0;
    a.jstride = 0;
    if (!J.d_jobs) {
        a.jmode = 0;
        a.jbase = J.inl.offset;
        return;
    }
    if (J.d_jidx || !J.h_jobs || J.njobs <= 0) return;
    const uint64_t b0 = J.h_jobs[0].offset;
    const uint64_t st = J.njobs > 1 ? J.h_jobs[1].offset - b0 : 0;
    for (int j = 0; j < J.njobs; ++j)
        if (J.h_jobs[j].offset != b0 + (uint64_t)j * st) return;
    a.jmode = 0;
    a.jbase = b0;
    a.jstride = st;
}

constexpr uint64_t kXcdMinBlocks = 8 * 256;  // eight blocks per CU

z2h_status launch_one_level(const Plan &P, void *states, const JobSet &J, int lev, int group,
                                   int rn_parts, bool force_plain, int kind, hipStream_t s,
                                   int kind_hint) {
    LevelArgs a;
    memset(&a, 0, sizeof a);
    a.states = states;
    a.jobs = J.d_jobs;
    a.job_inline = J.inl;
    a.geom = P.geom[group];
    a.lat = P.lat;
    a.level = lev;
    a.K = P.K;
    a.group = group;
    a.rn_parts = rn_parts;
    a.force_plain = force_plain ? 1 : 0;
    a.nt = P.nt;
    a.kind_hint = force_plain ? (int)kPlainH : kind_hint;
    a.njobs = J.njobs;
    a.jidx = J.d_jidx;
    if (!force_plain && J.d_btabs) {
        a.tabs = J.d_btabs;
        a.tab_stride = J.btab_stride;
    } else {
        a.tabs = force_plain ? nullptr : J.d_tabs;
        a.tab_lev0 = J.tab_lev0;
    }
    job_layout(J, a);
    const uint64_t nblocks = (uint64_t)J.njobs << a.geom.tiles_log2;
    if (nblocks > 0x7fffffffull) return fail(Z2H_ERR_UNSUPPORTED, "grid of %llu blocks", (unsigned long long)nblocks);
    // XCD-major order pays on streaming launches (many blocks per CU); a
    // launch of a few blocks per CU (a single small state) keeps the
    // hardware order, which measured slightly faster there
    a.xcd = ((P.xcd >> group) & 1) && nblocks >= kXcdMinBlocks;
    const size_t lds = lds_bytes(P, a.geom, a.geom.R);
    hipEvent_t e0, e1;
    timed_begin(s, e0, e1);
    hipError_t e = launch_level(P.c128, a.geom.R, a, (unsigned)nblocks, lds, s);
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "level kernel launch failed: %s", hipGetErrorString(e));
    timed_end(s, e0, e1, kind);
    return Z2H_OK;
}

// Unnormalized Walsh-Hadamard transform of every group (psi_1' preparation).
z2h_status full_transform(const Plan &P, void *states, const JobSet &J, hipStream_t s) {
    for (int gidx = 0; gidx < P.K; ++gidx) {
        z2h_status st = launch_one_level(P, states, J, 0, gidx, 0, true, 2, s);
        if (st) return st;
    }
    return Z2H_OK;
}

// Evolve the states of J through their level sequences.
z2h_status run_levels(const Plan &P, void *states, const JobSet &J, hipStream_t s) {
    int maxS = 0;
    bool any0 = false;
    for (int j = 0; j < J.njobs; ++j) {
        maxS = std::max(maxS, J.h_jobs[j].steps);
        if (J.h_jobs[j].order == 0) any0 = true;
    }
    if (maxS == 0) return Z2H_OK;
    if (P.K == 1) {
        ResidentArgs a;
        memset(&a, 0, sizeof a);
        a.states = states;
        a.jobs = J.d_jobs;
        a.job_inline = J.inl;
        a.geom = P.geom[0];
        a.lat = P.lat;
        a.job0 = 0;
        hipEvent_t e0, e1;
        timed_begin(s, e0, e1);
        hipError_t e = launch_resident(P.c128, a.geom.R, a, (unsigned)J.njobs, lds_bytes(P, a.geom, a.geom.R), s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "resident kernel launch failed: %s", hipGetErrorString(e));
        timed_end(s, e0, e1, 3);
        return Z2H_OK;
    }
    const int Pp = 2 * (P.K - 1);
    const int nlev = any0 ? Pp * (maxS + 1) + 1 : Pp * maxS + 1;
    const int parts0 = 1 << P.geom[0].tiles_log2;
    const bool big_parts = parts0 > 1024;
    // Levels of each job; jobs are ordered by decreasing level count, so the
    // jobs still running at a level are a prefix of the array.
    std::vector<int> jl(J.njobs);
    for (int j = 0; j < J.njobs; ++j) {
        const JobDev &h = J.h_jobs[j];
        jl[j] = h.steps <= 0 ? 0 : (h.order == 0 ? Pp * (h.steps + 1) + 1 : Pp * h.steps + 1);
        if (j > 0 && jl[j] > jl[j - 1])
            return fail(Z2H_ERR_INVALID, "internal: jobs not ordered by decreasing step count");
    }
    bool uses_norms = false;  // partials are written only where a renormalization or a trace reads them
    for (int j = 0; j < J.njobs; ++j) uses_norms = uses_norms || J.h_jobs[j].renorm || J.h_jobs[j].norm_trace;
    // a single inline job with table room: its phase tables are computed by
    // one launch per kTabChunk levels instead of by every workgroup
    const bool tabs = J.d_tabs && !J.d_jobs && J.njobs == 1;
    int tab_hi = 0, tab_lo = 0;
    int active = J.njobs;
    for (int lev = 0; lev < nlev; ++lev) {
        while (active > 0 && jl[active - 1] <= lev) --active;
        if (active == 0) break;
        if (tabs && lev >= tab_hi) {
            tab_lo = lev;
            tab_hi = std::min(nlev, lev + kTabChunk);
            TablesArgs ta;
            memset(&ta, 0, sizeof ta);
            ta.tabs = J.d_tabs;
            ta.job = J.inl;
            ta.lat = P.lat;
            ta.lev0 = tab_lo;
            ta.K = P.K;
            hipError_t e = launch_tables(P.c128, ta, (unsigned)(tab_hi - tab_lo), s);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "table kernel launch failed: %s", hipGetErrorString(e));
        }
        // the visited group is the same for every job; the kind may differ
        LevelOp op{};
        bool any_norm = false, uniform = true;
        for (int j = 0; j < active; ++j) {
            LevelOp o = level_op_host(lev, P.K, J.h_jobs[j].steps, J.h_jobs[j].k_begin, J.h_jobs[j].order);
            if (o.kind != kIdle) {
                if (op.kind == kIdle) op = o;
                else if (o.kind != op.kind) uniform = false;
                any_norm = any_norm || o.norm;
            } else {
                uniform = false;
            }
        }
        if (op.kind == kIdle) continue;
        JobSet Ja = J;
        Ja.njobs = active;
        if (!tabs) Ja.d_tabs = nullptr;
        Ja.tab_lev0 = tab_lo;
        z2h_status st = launch_one_level(P, states, Ja, lev, op.group, big_parts ? 1 : parts0, false,
                                         pass_kind_of(op), s, uniform ? (int)op.kind : -1);
        if (st) return st;
        if (big_parts && any_norm && uses_norms) {
            hipError_t e = launch_reduce_parts(J.d_jobs, J.inl, active, parts0, s);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "reduce kernel launch failed: %s", hipGetErrorString(e));
        }
    }
    return Z2H_OK;
}


int job_levels(const Plan &P, const JobDev &h) {
    const int Pp = 2 * (P.K - 1);
    return h.steps <= 0 ? 0 : (h.order == 0 ? Pp * (h.steps + 1) + 1 : Pp * h.steps + 1);
}

void pack_levels(const Plan &P, std::vector<JobDev> &h_jobs, int slots, PackedLevels &L) {
    const int Pp = 2 * (P.K - 1);
    const int nj = (int)h_jobs.size();
    std::vector<int> order(nj);
    for (int j = 0; j < nj; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return job_levels(P, h_jobs[x]) > job_levels(P, h_jobs[y]); });
    slots = std::max(1, std::min(slots, nj));
    std::vector<int64_t> end(slots, 0);
    int64_t total = 0;
    for (int j : order) {
        const int nl = job_levels(P, h_jobs[j]);
        h_jobs[j].lev0 = 0;
        if (nl == 0) continue;
        int best = 0;
        for (int q = 1; q < slots; ++q)
            if (end[q] < end[best]) best = q;
        h_jobs[j].lev0 = (int32_t)end[best];
        total = std::max<int64_t>(total, end[best] + nl);
        end[best] = (end[best] + nl + Pp - 1) / Pp * Pp;  // next start on a multiple of the passes per step
    }
    L.active.assign((size_t)total, {});
    for (int j = 0; j < nj; ++j) {
        const int nl = job_levels(P, h_jobs[j]);
        for (int l = 0; l < nl; ++l) L.active[(size_t)h_jobs[j].lev0 + l].push_back(j);
    }
    L.off.assign(L.active.size() + 1, 0);
    for (size_t l = 0; l < L.active.size(); ++l) L.off[l + 1] = L.off[l] + L.active[l].size();
    L.d_idx = nullptr;
}

z2h_status run_levels_packed(const Plan &P, void *states, const JobSet &J, const PackedLevels &L, hipStream_t s) {
    const int parts0 = 1 << P.geom[0].tiles_log2;
    if (parts0 > kReduceChunk)
        return fail(Z2H_ERR_UNSUPPORTED, "packed batches need at most %d norm partials per state", kReduceChunk);
    for (size_t lev = 0; lev < L.active.size(); ++lev) {
        const std::vector<int32_t> &act = L.active[lev];
        if (act.empty()) continue;
        LevelOp op{};
        bool uniform = true;
        for (int32_t j : act) {
            const JobDev &h = J.h_jobs[j];
            LevelOp o = level_op_host((int)lev - h.lev0, P.K, h.steps, h.k_begin, h.order);
            if (o.kind == kIdle) {
                uniform = false;
                continue;
            }
            if (op.kind == kIdle) op = o;
            else if (o.kind != op.kind) uniform = false;
            if (o.group != op.group) return fail(Z2H_ERR_INVALID, "internal: packed level %zu mixes groups", lev);
        }
        if (op.kind == kIdle) continue;
        JobSet Ja = J;
        Ja.njobs = (int)act.size();
        Ja.d_jidx = L.d_idx + L.off[lev];
        z2h_status st = launch_one_level(P, states, Ja, (int)lev, op.group, parts0, false, pass_kind_of(op), s,
                                         uniform ? (int)op.kind : -1);
        if (st) return st;
    }
    return Z2H_OK;
}


z2h_status run_observe(const Plan &P, const void *states, int njobs, const ObsBuffers &B,
                              const uint32_t *zl, int nz, const uint32_t *xl, int nx, hipStream_t s) {
    ObsArgs a;
    memset(&a, 0, sizeof a);
    a.lat = P.lat;
    for (int j = 0; j < nz; ++j) a.zloops[j] = zl[j];
    for (int j = 0; j < nx; ++j) a.xloops[j] = xl[j];
    a.nz = nz;
    a.nx = nx;
    int wZ = 0, wX = 0;
    for (int gi = 0; gi < P.K; ++gi) {
        a.geom = P.geom[gi];
        const int w = obs_workers(a.geom);
        a.src = gi == 0 ? states : B.scratch;
        a.src_off = gi == 0 ? B.src_off : B.dst_off;
        a.dst = gi == P.K - 1 ? nullptr : B.scratch;
        a.dst_off = B.dst_off;
        a.redZ = gi == 0;
        a.doH = 1;
        a.redX = gi == P.K - 1;
        a.part_z = gi == 0 ? B.partZ : nullptr;
        a.part_x = gi == P.K - 1 ? B.partX : nullptr;
        if (gi == 0) wZ = w;
        if (gi == P.K - 1) wX = w;
        hipError_t e = launch_obs(P.c128, a.geom.R, a, w, njobs, obs_lds_bytes(P, a.geom, a.geom.R), s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "observe kernel failed: %s", hipGetErrorString(e));
    }
    FinalArgs f;
    memset(&f, 0, sizeof f);
    f.partZ = B.partZ;
    f.partX = B.partX;
    f.nrecZ = wZ;
    f.nrecX = wX;
    f.n = P.n;
    f.H = B.H;
    for (int j = 0; j < 4; ++j) f.H_inline[j] = B.H_inline[j];
    f.out = B.out;
    f.out_index = B.out_index;
    hipError_t e = launch_obs_finalize(f, njobs, s);
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "observe finalize failed: %s", hipGetErrorString(e));
    return Z2H_OK;
}


size_t obs_records(const Plan &P) {
    return (size_t)obs_workers(P.geom[0]) + (size_t)obs_workers(P.geom[P.K - 1]);
}

// Doubles of norm partials per job: one per tile of the z pass, plus the
// first-stage slots when there are more partials than a pass reads.
size_t norm_parts(const Plan &P) {
    const size_t tiles = (size_t)1 << P.geom[0].tiles_log2;
    return tiles + (tiles > (size_t)kReduceChunk ? (tiles + kReduceChunk - 1) / kReduceChunk : 0);
}

// Phase tables of kTabChunk levels, after everything else in the evolve
// workspace, for multi-group plans whose phase passes run full-window
// kernels (",tables=0" in a schedule string turns them off).  The phase
// kernels fetch their block's share of a ready table ahead of the tile
// loads instead of computing sines and cosines in FP64 while the tile is
// in flight.
static bool tables_apply(const Plan &P) {
    return P.tables && P.K > 1 && P.geom[0].full && P.geom[P.K - 1].full;
}

size_t ws_tables_size(const Plan &P) {
    if (!tables_apply(P)) return 0;
    return align256((size_t)kTabChunk * (size_t)(P.nst + 1) * (size_t)(P.n + 1) * P.esize);
}

size_t ws_evolve_size(const Plan &P) {
    Carver c{nullptr, 0};
    c.take(sizeof(double) * norm_parts(P));
    return align256(c.off) + ws_tables_size(P);
}

size_t ws_observe_size(const Plan &P) {
    Carver c{nullptr, 0};
    if (P.K > 1) c.take(P.esize << P.n);
    c.take(sizeof(double) * kObsQ * obs_records(P));
    c.take(sizeof(double) * kObsQ);
    return align256(c.off);
}

}  // namespace rt
}  // namespace z2h

using namespace z2h;
using namespace z2h::rt;

// ------------------------------------------------------------------ C ABI

z2h_status z2h::rt::check_device_(const Plan &P) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(Z2H_ERR_HIP, "no HIP device");
    if (P.device >= 0 && dev != P.device)
        return fail(Z2H_ERR_INVALID, "current device %d differs from the plan's device %d", dev, P.device);
    return Z2H_OK;
}

z2h_status z2h::rt::check_loop_masks(const Plan &P, const uint64_t *m, int32_t cnt, const char *what,
                                   uint32_t *out) {
    if (cnt < 0 || cnt > Z2H_MAX_LOOPS) return fail(Z2H_ERR_INVALID, "%s count %d outside [0, %d]", what, cnt, Z2H_MAX_LOOPS);
    if (cnt && !m) return fail(Z2H_ERR_INVALID, "%s is NULL", what);
    for (int j = 0; j < cnt; ++j) {
        if (P.n < 64 && (m[j] >> P.n)) return fail(Z2H_ERR_INVALID, "%s[%d] has bits >= n", what, j);
        out[j] = (uint32_t)m[j];
    }
    return Z2H_OK;
}

extern "C" {

const char *z2h_version(void) { return "z2h 0.1 (gfx950)"; }

const char *z2h_last_error(void) { return g_err.c_str(); }

z2h_status z2h_link_bit(int32_t Lx, int32_t Ly, int32_t x, int32_t y, int32_t dir, int32_t *bit) {
    z2h_status st = check_lattice(Lx, Ly);
    if (st) return st;
    if (!bit) return fail(Z2H_ERR_INVALID, "bit is NULL");
    if (dir != 0 && dir != 1) return fail(Z2H_ERR_INVALID, "dir must be 0 or 1");
    *bit = link_bit(Lx, Ly, x, y, dir);
    return Z2H_OK;
}

z2h_status z2h_masks(int32_t Lx, int32_t Ly, uint64_t *stars, uint64_t *plaqs) {
    z2h_status st = check_lattice(Lx, Ly);
    if (st) return st;
    if (!stars || !plaqs) return fail(Z2H_ERR_INVALID, "mask arrays are NULL");
    build_masks(Lx, Ly, stars, plaqs);
    return Z2H_OK;
}

z2h_status z2h_plan_create(int32_t Lx, int32_t Ly, z2h_dtype dtype, int32_t max_tile_bits, z2h_plan **out) {
    try {
        if (!out) return fail(Z2H_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (dtype != Z2H_C64 && dtype != Z2H_C128) return fail(Z2H_ERR_INVALID, "bad dtype %d", dtype);
        z2h_plan *p = new (std::nothrow) z2h_plan;
        if (!p) return fail(Z2H_ERR_OOM, "out of host memory");
        z2h_status st = make_plan(Lx, Ly, dtype == Z2H_C128, max_tile_bits, p->P, 1);
        if (st) {
            delete p;
            return st;
        }
        p->P.device = -1;
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
            int dev = 0;
            if (hipGetDevice(&dev) == hipSuccess) p->P.device = dev;
        }
        *out = p;
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in plan creation");
    }
}

void z2h_plan_destroy(z2h_plan *plan) { delete plan; }

z2h_status z2h_plan_sizes(const z2h_plan *plan, size_t *state_bytes, size_t *ws_evolve_bytes,
                          size_t *ws_observe_bytes, size_t *ws_adjoint_bytes) {
    if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
    const Plan &P = plan->P;
    if (state_bytes) *state_bytes = P.esize << P.n;
    if (ws_evolve_bytes) *ws_evolve_bytes = ws_evolve_size(P);
    if (ws_observe_bytes) *ws_observe_bytes = ws_observe_size(P);
    if (ws_adjoint_bytes) *ws_adjoint_bytes = ws_adjoint_size(P);
    return Z2H_OK;
}

z2h_status z2h_plan_info(const z2h_plan *plan, int32_t *n, int32_t *groups, int32_t *passes_per_step,
                         int32_t *tile_bits) {
    if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
    const Plan &P = plan->P;
    if (n) *n = P.n;
    if (groups) *groups = P.K;
    if (passes_per_step) *passes_per_step = P.K == 1 ? 0 : 2 * (P.K - 1);
    if (tile_bits) *tile_bits = P.geom[0].m;
    return Z2H_OK;
}

z2h_status z2h_plan_describe(const z2h_plan *plan, char *buf, size_t len) {
    if (!plan || !buf || len == 0) return fail(Z2H_ERR_INVALID, "NULL argument");
    const Plan &P = plan->P;
    std::string s = "{\"n\": " + std::to_string(P.n) + ", \"R\": " + std::to_string(P.geom[0].R) +
                    ", \"K\": " + std::to_string(P.K) + ", \"c128\": " + (P.c128 ? "1" : "0") + ", \"nt\": " + std::to_string(P.nt) +
                    ", \"xcd\": " + std::to_string(P.xcd) + ", \"tables\": " + std::to_string(P.tables) +
                    ", \"groups\": [";
    for (int j = 0; j < P.K; ++j) {
        const GroupGeom &g = P.geom[j];
        s += j ? ", " : "";
        s += "{\"m\": " + std::to_string(g.m) + ", \"c\": " + std::to_string(g.c) +
             ", \"b0\": " + std::to_string(g.b0) + ", \"hi\": " + std::to_string(g.hi) +
             ", \"b1\": " + std::to_string(g.b1) + ", \"x0\": " + std::to_string(g.x0) +
             ", \"x1\": " + std::to_string(g.x1) + ", \"tiles_log2\": " + std::to_string(g.tiles_log2) +
             ", \"p\": [";
        for (int l = 0; l < g.nlay; ++l) s += (l ? ", " : "") + std::to_string(g.p[l]);
        s += "], \"blo\": [";
        for (int l = 0; l < g.nlay; ++l) s += (l ? ", " : "") + std::to_string(g.blo[l]);
        s += "], \"bhi\": [";
        for (int l = 0; l < g.nlay; ++l) s += (l ? ", " : "") + std::to_string(g.bhi[l]);
        s += "], \"lds_bytes\": " + std::to_string(lds_bytes(P, g, g.R)) + ", \"R\": " + std::to_string(g.R) +
             ", \"full\": " + std::to_string(g.full) + ", \"pair\": " + std::to_string(g.pair >= 2 ? 2 : 1) +
             ", \"cx\": " + std::to_string(g.cx) +
             ", \"lds_blk\": " + std::to_string(g.lds_blk) + "}";
    }
    s += "]}";
    if (s.size() + 1 > len) return fail(Z2H_ERR_INVALID, "buffer of %zu bytes, %zu needed", len, s.size() + 1);
    memcpy(buf, s.c_str(), s.size() + 1);
    return Z2H_OK;
}

z2h_status z2h_state_init(const z2h_plan *plan, void *d_state, z2h_init kind, void *stream) {
    if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
    z2h_status st = validate_state_ptr(d_state, "d_state");
    if (st) return st;
    if (kind < Z2H_INIT_PSI1 || kind > Z2H_INIT_PLUS) return fail(Z2H_ERR_INVALID, "bad init kind %d", kind);
    const Plan &P = plan->P;
    if ((st = check_device_(P))) return st;
    hipStream_t s = (hipStream_t)stream;
    InitArgs a;
    memset(&a, 0, sizeof a);
    a.states = d_state;
    a.lat = P.lat;
    a.one_job = init_job(P, kind, 0);
    hipError_t e = launch_init(P.c128, a, 1, s);
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "init kernel failed: %s", hipGetErrorString(e));
    if (kind == Z2H_INIT_PSI1P) {
        // psi_1' = H^n (star-even superposition in the Hadamard basis)
        JobSet J;
        memset(&J, 0, sizeof J);
        J.njobs = 1;
        return full_transform(P, d_state, J, s);
    }
    return Z2H_OK;
}

z2h_status z2h_evolve(const z2h_plan *plan, void *d_state, void *d_ws, size_t ws_bytes,
                      const z2h_schedule *sched, double *d_norms, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        z2h_status st = validate_state_ptr(d_state, "d_state");
        if (st) return st;
        if ((st = validate_schedule(P, sched))) return st;
        if (!d_ws) return fail(Z2H_ERR_INVALID, "d_ws is NULL");
        const bool arrays = sched->sZ || sched->sX;
        if (arrays) {
            for (int64_t k = 0; k < sched->steps; ++k) {
                if ((sched->sZ && !std::isfinite(sched->sZ[k])) || (sched->sX && !std::isfinite(sched->sX[k])))
                    return fail(Z2H_ERR_INVALID, "schedule value at step %lld not finite", (long long)k);
            }
        }
        size_t need = ws_evolve_size(P);
        if (arrays) need += align256(sizeof(double) * 2 * (size_t)sched->steps) + 256;
        if (ws_bytes < need)
            return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if ((st = check_device_(P))) return st;
        hipStream_t s = (hipStream_t)stream;
        Carver c{(char *)d_ws, 0};
        JobSet J;
        memset(&J, 0, sizeof J);
        J.inl = make_job(sched, 0);
        J.inl.norm_part = (double *)c.take(sizeof(double) * norm_parts(P));
        J.inl.norm_trace = d_norms;
        if (arrays) {
            double *dz = (double *)c.take(sizeof(double) * sched->steps);
            double *dx = (double *)c.take(sizeof(double) * sched->steps);
            if (sched->sZ) HIP_TRY(hipMemcpyAsync(dz, sched->sZ, sizeof(double) * sched->steps, hipMemcpyHostToDevice, s));
            if (sched->sX) HIP_TRY(hipMemcpyAsync(dx, sched->sX, sizeof(double) * sched->steps, hipMemcpyHostToDevice, s));
            // the host arrays may be reused as soon as this call returns
            HIP_TRY(hipStreamSynchronize(s));
            J.inl.sZ = sched->sZ ? dz : nullptr;
            J.inl.sX = sched->sX ? dx : nullptr;
        }
        if (ws_tables_size(P)) J.d_tabs = c.take(ws_tables_size(P));
        J.h_jobs = &J.inl;
        J.njobs = 1;
        return run_levels(P, d_state, J, s);
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_evolve");
    }
}

z2h_status z2h_observe(const z2h_plan *plan, const void *d_state, void *d_ws, size_t ws_bytes,
                       const z2h_couplings *H, const uint64_t *zmasks, int32_t nz, const uint64_t *xmasks,
                       int32_t nx, z2h_obs *h_out, double *d_out, void *stream) {
    try {
        if (!plan) return fail(Z2H_ERR_INVALID, "plan is NULL");
        const Plan &P = plan->P;
        z2h_status st = validate_state_ptr(d_state, "d_state");
        if (st) return st;
        if (!H) return fail(Z2H_ERR_INVALID, "H is NULL");
        if (!d_ws) return fail(Z2H_ERR_INVALID, "d_ws is NULL");
        if (!h_out && !d_out) return fail(Z2H_ERR_INVALID, "no output requested");
        uint32_t zl[Z2H_MAX_LOOPS], xl[Z2H_MAX_LOOPS];
        if ((st = check_loop_masks(P, zmasks, nz, "zmasks", zl))) return st;
        if ((st = check_loop_masks(P, xmasks, nx, "xmasks", xl))) return st;
        const size_t need = ws_observe_size(P);
        if (ws_bytes < need) return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        if ((st = check_device_(P))) return st;
        hipStream_t s = (hipStream_t)stream;
        Carver c{(char *)d_ws, 0};
        ObsBuffers B;
        memset(&B, 0, sizeof B);
        if (P.K > 1) B.scratch = c.take(P.esize << P.n);
        const size_t wz = obs_workers(P.geom[0]);
        double *parts = (double *)c.take(sizeof(double) * kObsQ * obs_records(P));
        B.partZ = parts;
        B.partX = parts + wz * kObsQ;
        double *outbuf = (double *)c.take(sizeof(double) * kObsQ);
        B.out = d_out ? d_out : outbuf;
        B.H_inline[0] = H->JA;
        B.H_inline[1] = H->JB;
        B.H_inline[2] = H->hx;
        B.H_inline[3] = H->hz;
        if ((st = run_observe(P, d_state, 1, B, zl, nz, xl, nx, s))) return st;
        if (h_out) {
            double tmp[kObsQ];
            HIP_TRY(hipMemcpyAsync(tmp, B.out, sizeof tmp, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            memcpy(h_out, tmp, sizeof(z2h_obs));
            if (!std::isfinite(h_out->norm) || !std::isfinite(h_out->energy))
                return fail(Z2H_ERR_NUMERIC, "non-finite norm (%g) or energy (%g)", h_out->norm, h_out->energy);
        }
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_observe");
    }
}

z2h_status z2h_timing_enable(int32_t on) {
    t_timing = on != 0;
    return Z2H_OK;
}

z2h_status z2h_timing_read(int64_t counts[4], double ms[4]) {
    if (!counts || !ms) return fail(Z2H_ERR_INVALID, "NULL output");
    for (int k = 0; k < 4; ++k) {
        counts[k] = 0;
        ms[k] = 0;
    }
    z2h_status st = Z2H_OK;
    for (auto &L : t_launches) {
        float x = 0;
        if (hipEventSynchronize(L.b) != hipSuccess || hipEventElapsedTime(&x, L.a, L.b) != hipSuccess)
            st = fail(Z2H_ERR_HIP, "event timing failed");
        counts[L.kind] += 1;
        ms[L.kind] += x;
        t_pool.push_back(L.a);
        t_pool.push_back(L.b);
    }
    t_launches.clear();
    return st;
}

}  // extern "C"
