// Gate-level circuits of Sec. III (the Trotter step with an ancilla) and of
// Eqs. (ini1), (ini2) (state preparation), and their execution on the
// device: one launch per gate, or groups of consecutive gates applied in
// LDS tiles by one pass each.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "z2h_runtime.h"
#include "z2h_solvers.h"

using namespace z2h;
using namespace z2h::rt;

namespace {

constexpr int kMaxCircuitQubits = 34;

z2h_gate gate(int kind, int q0, int q1 = 0, double theta = 0.0) {
    z2h_gate g;
    g.kind = kind;
    g.q0 = q0;
    g.q1 = q1;
    g.reserved = 0;
    g.theta = theta;
    return g;
}

std::vector<int> bits_of(uint64_t mask) {
    std::vector<int> b;
    for (int l = 0; l < 64; ++l)
        if (mask >> l & 1) b.push_back(l);
    return b;
}

// exp(i (-theta/2) Z_mask) through the ancilla: the CNOTs copy the parity of
// the masked links onto the ancilla (in |0>), R_z(theta) acts on it, and the
// same CNOTs clear it again.
void parity_gadget(std::vector<z2h_gate> &c, uint64_t mask, int anc, double theta) {
    const std::vector<int> ls = bits_of(mask);
    for (int l : ls) c.push_back(gate(Z2H_GATE_CNOT, l, anc));
    c.push_back(gate(Z2H_GATE_RZ, anc, 0, theta));
    for (int l : ls) c.push_back(gate(Z2H_GATE_CNOT, l, anc));
}

// Half of the stabilizer layer, exp(-i H_2 dt/2): per plaquette
// exp(i JB B_p dt/2) = U_1 R_z(-JB dt)_a U_1^dagger, then per star
// exp(i JA A_v dt/2) = U_2^dagger R_z(-JA dt)_a U_2 with U_2 the star's
// Hadamards followed by its CNOTs.
void stabilizer_half(std::vector<z2h_gate> &c, int nv, const uint64_t *st, const uint64_t *pl, int anc,
                     double JA, double JB, double dt) {
    for (int p = 0; p < nv; ++p) parity_gadget(c, pl[p], anc, -JB * dt);
    for (int v = 0; v < nv; ++v) {
        const std::vector<int> ls = bits_of(st[v]);
        for (int l : ls) c.push_back(gate(Z2H_GATE_H, l));
        parity_gadget(c, st[v], anc, -JA * dt);
        for (int l : ls) c.push_back(gate(Z2H_GATE_H, l));
    }
}

void rotation_layer(std::vector<z2h_gate> &c, int n, int kind, double theta) {
    for (int l = 0; l < n; ++l) c.push_back(gate(kind, l, 0, theta));
}

std::vector<z2h_gate> step_circuit(int Lx, int Ly, const z2h_couplings &cx, const z2h_couplings &cz, double dt,
                                   int order) {
    uint64_t st[kMaxStab], pl[kMaxStab];
    build_masks(Lx, Ly, st, pl);
    const int n = 2 * Lx * Ly, nv = Lx * Ly, anc = n;
    std::vector<z2h_gate> c;
    c.reserve((size_t)(3 * n + 2 * 26 * nv));
    if (order == 0) {
        // exp(-iH_1 dt/2) exp(-iH_2 dt/2) exp(-iH_3 dt) exp(-iH_2 dt/2) exp(-iH_1 dt/2), Eq. (gate1)
        rotation_layer(c, n, Z2H_GATE_RX, -cx.hx * dt);
        stabilizer_half(c, nv, st, pl, anc, cx.JA, cz.JB, dt);
        rotation_layer(c, n, Z2H_GATE_RZ, -2.0 * cz.hz * dt);
        stabilizer_half(c, nv, st, pl, anc, cx.JA, cz.JB, dt);
        rotation_layer(c, n, Z2H_GATE_RX, -cx.hx * dt);
    } else {
        rotation_layer(c, n, Z2H_GATE_RZ, -cz.hz * dt);
        stabilizer_half(c, nv, st, pl, anc, cx.JA, cz.JB, dt);
        rotation_layer(c, n, Z2H_GATE_RX, -2.0 * cx.hx * dt);
        stabilizer_half(c, nv, st, pl, anc, cx.JA, cz.JB, dt);
        rotation_layer(c, n, Z2H_GATE_RZ, -cz.hz * dt);
    }
    return c;
}

std::vector<z2h_gate> prep_circuit(int Lx, int Ly, int which) {
    uint64_t st[kMaxStab], pl[kMaxStab];
    build_masks(Lx, Ly, st, pl);
    const int n = 2 * Lx * Ly, nv = Lx * Ly, anc = n;
    std::vector<z2h_gate> c;
    if (which == Z2H_INIT_PSI1) {
        for (int l = 0; l < n; ++l) c.push_back(gate(Z2H_GATE_H, l));
        for (int p = 0; p < nv; ++p) {
            const std::vector<int> ls = bits_of(pl[p]);
            for (int l : ls) c.push_back(gate(Z2H_GATE_CNOT, l, anc));
            c.push_back(gate(Z2H_GATE_PROJ0, anc));
            for (int l : ls) c.push_back(gate(Z2H_GATE_CNOT, l, anc));
        }
    } else {
        for (int v = 0; v < nv; ++v) {
            const std::vector<int> ls = bits_of(st[v]);
            for (int l : ls) c.push_back(gate(Z2H_GATE_H, l));
            for (int l : ls) c.push_back(gate(Z2H_GATE_CNOT, l, anc));
            c.push_back(gate(Z2H_GATE_PROJ0, anc));
            for (int l : ls) c.push_back(gate(Z2H_GATE_CNOT, l, anc));
            for (int l : ls) c.push_back(gate(Z2H_GATE_H, l));
        }
    }
    c.push_back(gate(Z2H_GATE_NORM, 0));
    return c;
}

z2h_status copy_out(const std::vector<z2h_gate> &c, z2h_gate *out, int32_t cap, int32_t *count) {
    if (!count) return fail(Z2H_ERR_INVALID, "count is NULL");
    *count = (int32_t)c.size();
    if (!out || cap < (int32_t)c.size())
        return fail(Z2H_ERR_WORKSPACE, "%zu gates, room for %d", c.size(), cap);
    std::copy(c.begin(), c.end(), out);
    return Z2H_OK;
}

// Device form of a gate (2x2 matrix of a one-qubit gate in FP64).
GateDev device_gate(const z2h_gate &g, int q0, int q1) {
    GateDev d;
    memset(&d, 0, sizeof d);
    d.kind = g.kind;
    d.q0 = q0;
    d.q1 = q1;
    const double h = 0.5 * g.theta, c = std::cos(h), s = std::sin(h);
    if (g.kind == Z2H_GATE_H) {
        const double r = 1.0 / std::sqrt(2.0);
        const double m[8] = {r, 0, r, 0, r, 0, -r, 0};
        memcpy(d.m, m, sizeof m);
    } else if (g.kind == Z2H_GATE_RX) {  // exp(-i theta X / 2)
        const double m[8] = {c, 0, 0, -s, 0, -s, c, 0};
        memcpy(d.m, m, sizeof m);
    } else if (g.kind == Z2H_GATE_RZ) {  // exp(-i theta Z / 2)
        const double m[8] = {c, -s, 0, 0, 0, 0, c, s};
        memcpy(d.m, m, sizeof m);
    }
    return d;
}

// Append gate x, acting on register bits b0 (and b1, a CNOT's target), in
// the register kernels' form.  A CNOT right after another with the same
// target (both at index >= from, i.e. in one phase) is composed into it:
// the target flips with the parity of the XOR of their control masks, and
// a mask that cancels to zero drops the gate.  Hadamards are counted for
// the group's final scale.
static void append_reg_gate(GateDev *out, int &n, int from, const z2h_gate &x, int b0, int b1, int &nh) {
    if (x.kind == Z2H_GATE_CNOT) {
        if (n > from && out[n - 1].kind == Z2H_GATE_CNOT && out[n - 1].q1 == b1) {
            out[n - 1].q0 ^= 1 << b0;
            if (out[n - 1].q0 == 0) --n;
            return;
        }
        GateDev d;
        memset(&d, 0, sizeof d);
        d.kind = Z2H_GATE_CNOT;
        d.q0 = 1 << b0;
        d.q1 = b1;
        out[n++] = d;
        return;
    }
    if (x.kind == Z2H_GATE_H) ++nh;
    out[n++] = device_gate(x, b0, 0);
}

// 2^(-h/2): the factor that the unscaled Hadamard butterflies leave out.
static double hadamard_scale(int nh) { return std::ldexp(nh % 2 ? 1.0 / std::sqrt(2.0) : 1.0, -(nh / 2)); }

z2h_status check_gates(int nq, const z2h_gate *g, int ng) {
    for (int i = 0; i < ng; ++i) {
        const int k = g[i].kind;
        if (k < Z2H_GATE_H || k > Z2H_GATE_NORM) return fail(Z2H_ERR_INVALID, "gate %d: kind %d", i, k);
        if (k == Z2H_GATE_NORM) continue;
        if (g[i].q0 < 0 || g[i].q0 >= nq) return fail(Z2H_ERR_INVALID, "gate %d: qubit %d outside [0, %d)", i, g[i].q0, nq);
        if (k == Z2H_GATE_CNOT && (g[i].q1 < 0 || g[i].q1 >= nq || g[i].q1 == g[i].q0))
            return fail(Z2H_ERR_INVALID, "gate %d: CNOT target %d", i, g[i].q1);
        if (!std::isfinite(g[i].theta)) return fail(Z2H_ERR_INVALID, "gate %d: angle not finite", i);
    }
    return Z2H_OK;
}

int gate_parts(int nq) {
    const uint64_t b = ((1ull << nq) + 255) / 256;
    return (int)std::min<uint64_t>(b, (uint64_t)kGateBlocksMax);
}

// One launch per gate.
z2h_status run_unfused(int nq, bool c128, void *st, double *parts, const z2h_gate *g, int ng, hipStream_t s) {
    for (int i = 0; i < ng; ++i) {
        hipError_t e;
        if (g[i].kind == Z2H_GATE_NORM)
            e = launch_normalize(c128, st, nq, parts, gate_parts(nq), s);
        else
            e = launch_gate(c128, st, nq, device_gate(g[i], g[i].q0, g[i].q1), s);
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "gate %d failed: %s", i, hipGetErrorString(e));
    }
    return Z2H_OK;
}

// Qubits a gate acts on, as a bit mask.
static uint64_t gate_mask(const z2h_gate &x) {
    return (1ull << x.q0) | (x.kind == Z2H_GATE_CNOT ? 1ull << x.q1 : 0ull);
}

// Groups of the gates g[lo, hi) (no renormalisation among them) for the
// fused executors.  Each group is built by one scan over the gates not yet
// placed, in their order: a gate joins if no skipped earlier gate shares a
// qubit with it and the union of the group's qubits and `base` stays within
// `limit` qubits.  A gate that does not join blocks its qubits for the rest
// of the scan.  So a gate only ever moves ahead of gates on other qubits,
// with which it commutes, and each group keeps the gates' relative order.
// Rotation layers thereby join the gadget groups that touch their qubits.
static std::vector<std::vector<int>> gate_groups(const z2h_gate *g, int lo, int hi, int limit, uint64_t base) {
    std::vector<int> rest, left;
    for (int i = lo; i < hi; ++i) rest.push_back(i);
    std::vector<std::vector<int>> out;
    while (!rest.empty()) {
        std::vector<int> grp;
        uint64_t used = base, blocked = 0;
        left.clear();
        for (int i : rest) {
            const uint64_t m = gate_mask(g[i]);
            if (!(m & blocked) && __builtin_popcountll(used | m) <= limit && (int)grp.size() < kFuseMaxGates) {
                grp.push_back(i);
                used |= m;
            } else {
                blocked |= m;
                left.push_back(i);
            }
        }
        out.push_back(std::move(grp));
        rest.swap(left);
    }
    return out;
}

// The passes of a fused run: each maximal run of gates between
// renormalisations is grouped by gate_groups; a renormalisation is a pass of
// its own (a group holding just that gate).
static std::vector<std::vector<int>> plan_passes(const z2h_gate *g, int ng, int limit, uint64_t base) {
    std::vector<std::vector<int>> plan;
    int lo = 0;
    for (int i = 0; i <= ng; ++i) {
        if (i < ng && g[i].kind != Z2H_GATE_NORM) continue;
        for (std::vector<int> &grp : gate_groups(g, lo, i, limit, base)) plan.push_back(std::move(grp));
        if (i < ng) plan.push_back({i});
        lo = i + 1;
    }
    return plan;
}

// Run the plan: each group goes to `pass` (group indices, union of the
// group's qubits); renormalisations run in between.
template <typename Pass>
static z2h_status run_grouped(int nq, bool c128, void *st, double *parts, const z2h_gate *g, int ng, int limit,
                              uint64_t base, hipStream_t s, Pass pass) {
    for (const std::vector<int> &grp : plan_passes(g, ng, limit, base)) {
        if (grp.size() == 1 && g[grp[0]].kind == Z2H_GATE_NORM) {
            hipError_t e = launch_normalize(c128, st, nq, parts, gate_parts(nq), s);
            if (e != hipSuccess) return fail(Z2H_ERR_HIP, "normalisation failed: %s", hipGetErrorString(e));
            continue;
        }
        uint64_t used = 0;
        for (int j : grp) used |= gate_mask(g[j]);
        z2h_status st_ = pass(grp, used);
        if (st_) return st_;
    }
    return Z2H_OK;
}

// Qubit limit and always-local qubits of a fused executor (fuse 1: tile
// groups, fuse 2: register groups) for nq qubits, after the fallbacks of
// run_fused and run_reg; limit 0 means gate by gate.
static void fused_limits(int nq, bool c128, int fuse, int *limit, uint64_t *base) {
    if (fuse == 2 && nq >= kRegBits + 6) {
        *limit = kRegBits;
        *base = 0;
        return;
    }
    if (fuse >= 1 && nq >= kRegBits + 1) {
        const int mloc = std::min(nq, c128 ? 12 : 13);
        *limit = mloc;
        *base = (1ull << std::min(4, mloc)) - 1ull;
        return;
    }
    *limit = 0;
    *base = 0;
}

// One tile-group pass: the tile holds the group's qubits `used`, the four
// lowest qubits (coalesced rows of 16 amplitudes) and, as padding, the
// lowest remaining qubits, mloc in all.  Within the group, consecutive gates
// form a phase while the union of their local bits fits the kRegBits
// register bits; a phase's layout is padded with the highest local bits, so
// a phase on the top local bits needs no change of layout.
static z2h_status tile_pass(int nq, bool c128, void *st, const z2h_gate *g, const std::vector<int> &group,
                            uint64_t used, hipStream_t s) {
    int mloc;
    uint64_t base;
    fused_limits(nq, c128, 1, &mloc, &base);
    std::vector<char> in(nq, 0);
    int nin = 0;
    for (int q = 0; q < nq; ++q)
        if ((used | base) >> q & 1ull) {
            in[q] = 1;
            ++nin;
        }
    for (int q = 0; q < nq && nin < mloc; ++q)
        if (!in[q]) {
            in[q] = 1;
            ++nin;
        }
    FusedArgs a;
    memset(&a, 0, sizeof a);
    a.state = st;
    a.nq = nq;
    a.m = mloc;
    int loc[kMaxCircuitQubits];
    int nl = 0, nc = 0;
    for (int q = 0; q < nq; ++q) {
        if (in[q]) {
            loc[q] = nl;
            a.lq[nl++] = q;
        } else {
            a.cq[nc++] = q;
        }
    }
    const int ng_src = (int)group.size();
    std::vector<int> bits;
    int first = 0, nd = 0, nh = 0;
    auto close = [&](int end) {
        std::vector<int> lay = bits;
        for (int b = mloc - 1; (int)lay.size() < kRegBits; --b)
            if (std::find(lay.begin(), lay.end(), b) == lay.end()) lay.push_back(b);
        std::sort(lay.begin(), lay.end());
        uint32_t code = 0;
        int rb[16];
        for (int b = 0; b < kRegBits; ++b) {
            code |= (uint32_t)lay[b] << (4 * b);
            rb[lay[b]] = b;
        }
        const int from = nd;
        for (int i = first; i < end; ++i) {
            const z2h_gate &x = g[group[i]];
            append_reg_gate(a.gates, nd, from, x, rb[loc[x.q0]], x.kind == Z2H_GATE_CNOT ? rb[loc[x.q1]] : 0, nh);
        }
        if (nd > from) a.phase[a.nphase++] = code | (uint32_t)nd << 24;
        first = end;
        bits.clear();
    };
    for (int i = 0; i < ng_src; ++i) {
        const z2h_gate &x = g[group[i]];
        const int b0 = loc[x.q0], b1 = x.kind == Z2H_GATE_CNOT ? loc[x.q1] : b0;
        const bool h0 = std::find(bits.begin(), bits.end(), b0) != bits.end();
        const bool h1 = b1 == b0 || std::find(bits.begin(), bits.end(), b1) != bits.end();
        if ((int)bits.size() + !h0 + !h1 > kRegBits) close(i);
        if (std::find(bits.begin(), bits.end(), b0) == bits.end()) bits.push_back(b0);
        if (std::find(bits.begin(), bits.end(), b1) == bits.end()) bits.push_back(b1);
    }
    close(ng_src);
    a.ngates = nd;
    a.scale = hadamard_scale(nh);
    hipError_t e = nd ? launch_fused(c128, a, s) : hipSuccess;
    if (e != hipSuccess) return fail(Z2H_ERR_HIP, "fused gate pass failed: %s", hipGetErrorString(e));
    return Z2H_OK;
}

// Tile groups: gate_groups with the tile width as the limit and the four
// lowest qubits always in the tile.
z2h_status run_fused(int nq, bool c128, void *st, double *parts, const z2h_gate *g, int ng, hipStream_t s) {
    if (nq < kRegBits + 1) return run_unfused(nq, c128, st, parts, g, ng, s);
    int mloc;
    uint64_t base;
    fused_limits(nq, c128, 1, &mloc, &base);
    auto pass = [&](const std::vector<int> &group, uint64_t used) -> z2h_status {
        return tile_pass(nq, c128, st, g, group, used, s);
    };
    return run_grouped(nq, c128, st, parts, g, ng, mloc, base, s, pass);
}

// Register groups: gate_groups on at most kRegBits qubits, applied by one
// pass in which every thread holds the amplitudes that differ in those
// qubits.  The group's qubit set is padded with the highest remaining qubits
// so that the 256 threads of a block cover the lowest ones (coalesced
// access).  States of fewer than kRegBits + 6 qubits use tile groups instead.
z2h_status run_reg(int nq, bool c128, void *st, double *parts, const z2h_gate *g, int ng, hipStream_t s) {
    if (nq < kRegBits + 6) return run_fused(nq, c128, st, parts, g, ng, s);
    const int nt = std::min(8, nq - kRegBits);
    auto pass = [&](const std::vector<int> &group, uint64_t used) -> z2h_status {
        // With qubits 0, 1 and 2 in the registers, a wave's lanes would lie
        // at least 64 B apart and every line would be assembled from several
        // loads and stores; the tile kernel applies such a group with
        // coalesced rows instead (the group also fits its tile).
        if ((used & 7ull) == 7ull) return tile_pass(nq, c128, st, g, group, used, s);
        std::vector<char> in(nq, 0);
        std::vector<int> U;
        for (int q = 0; q < nq; ++q)
            if (used >> q & 1ull) {
                in[q] = 1;
                U.push_back(q);
            }
        for (int q = nq - 1; (int)U.size() < kRegBits; --q)
            if (!in[q]) {
                in[q] = 1;
                U.push_back(q);
            }
        RegArgs a;
        memset(&a, 0, sizeof a);
        a.state = st;
        a.nq = nq;
        a.nt = nt;
        int loc[kMaxCircuitQubits];
        for (int i = 0; i < kRegBits; ++i) {
            a.rq[i] = U[i];
            loc[U[i]] = i;
        }
        int k = 0, c = 0;
        for (int q = 0; q < nq; ++q) {
            if (in[q]) continue;
            if (k < nt)
                a.tq[k++] = q;
            else
                a.cq[c++] = q;
        }
        int nd = 0, nh = 0;
        for (int i = 0; i < (int)group.size(); ++i) {
            const z2h_gate &x = g[group[i]];
            append_reg_gate(a.gates, nd, 0, x, loc[x.q0], x.kind == Z2H_GATE_CNOT ? loc[x.q1] : 0, nh);
        }
        a.ngates = nd;
        a.scale = hadamard_scale(nh);
        hipError_t e = nd ? launch_reg(c128, a, s) : hipSuccess;
        if (e != hipSuccess) return fail(Z2H_ERR_HIP, "register gate pass failed: %s", hipGetErrorString(e));
        return Z2H_OK;
    };
    return run_grouped(nq, c128, st, parts, g, ng, kRegBits, 0ull, s, pass);
}

z2h_status run_gates(int nq, z2h_dtype dtype, void *d_state, void *d_ws, size_t ws_bytes, const z2h_gate *gates,
                     int ng, int fuse, hipStream_t s) {
    if (nq < 2 || nq > kMaxCircuitQubits) return fail(Z2H_ERR_INVALID, "nq = %d outside [2, %d]", nq, kMaxCircuitQubits);
    if (dtype != Z2H_C64 && dtype != Z2H_C128) return fail(Z2H_ERR_INVALID, "unknown dtype %d", dtype);
    if (fuse < 0 || fuse > 2) return fail(Z2H_ERR_INVALID, "fuse must be 0, 1 or 2");
    if (ng < 0 || (ng > 0 && !gates)) return fail(Z2H_ERR_INVALID, "gate list");
    z2h_status st = validate_state_ptr(d_state, "d_state");
    if (st) return st;
    if (!d_ws) return fail(Z2H_ERR_INVALID, "d_ws is NULL");
    if (ws_bytes < sizeof(double) * (size_t)gate_parts(nq))
        return fail(Z2H_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes,
                    sizeof(double) * (size_t)gate_parts(nq));
    if ((st = check_gates(nq, gates, ng))) return st;
    const bool c128 = dtype == Z2H_C128;
    if (fuse == 2) return run_reg(nq, c128, d_state, (double *)d_ws, gates, ng, s);
    return fuse ? run_fused(nq, c128, d_state, (double *)d_ws, gates, ng, s)
                : run_unfused(nq, c128, d_state, (double *)d_ws, gates, ng, s);
}

}  // namespace

extern "C" {

z2h_status z2h_circuit_step(int32_t Lx, int32_t Ly, const z2h_couplings *cx, const z2h_couplings *cz, double dt,
                            int32_t order, z2h_gate *out, int32_t cap, int32_t *count) {
    try {
        z2h_status st = check_lattice(Lx, Ly);
        if (st) return st;
        if (2 * Lx * Ly + 1 > kMaxCircuitQubits) return fail(Z2H_ERR_UNSUPPORTED, "%d links plus the ancilla", 2 * Lx * Ly);
        if (!cx || !cz) return fail(Z2H_ERR_INVALID, "couplings NULL");
        if (order != 0 && order != 1) return fail(Z2H_ERR_INVALID, "order must be 0 or 1");
        return copy_out(step_circuit(Lx, Ly, *cx, *cz, dt, order), out, cap, count);
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_circuit_step");
    }
}

z2h_status z2h_circuit_prep(int32_t Lx, int32_t Ly, int32_t which, z2h_gate *out, int32_t cap, int32_t *count) {
    try {
        z2h_status st = check_lattice(Lx, Ly);
        if (st) return st;
        if (2 * Lx * Ly + 1 > kMaxCircuitQubits) return fail(Z2H_ERR_UNSUPPORTED, "%d links plus the ancilla", 2 * Lx * Ly);
        if (which != Z2H_INIT_PSI1 && which != Z2H_INIT_PSI1P)
            return fail(Z2H_ERR_INVALID, "which must be Z2H_INIT_PSI1 or Z2H_INIT_PSI1P");
        return copy_out(prep_circuit(Lx, Ly, which), out, cap, count);
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_circuit_prep");
    }
}

size_t z2h_gates_ws_bytes(int32_t nq) {
    if (nq < 2 || nq > kMaxCircuitQubits) return 0;
    return align256(sizeof(double) * (size_t)gate_parts(nq));
}

z2h_status z2h_gates_run(int32_t nq, z2h_dtype dtype, void *d_state, void *d_ws, size_t ws_bytes,
                         const z2h_gate *gates, int32_t ngates, int32_t fuse, void *stream) {
    try {
        return run_gates(nq, dtype, d_state, d_ws, ws_bytes, gates, ngates, fuse, (hipStream_t)stream);
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_gates_run");
    }
}

z2h_status z2h_gates_schedule(int32_t nq, z2h_dtype dtype, const z2h_gate *gates, int32_t ngates, int32_t fuse,
                              int32_t *pass_of, int32_t *npasses) {
    try {
        if (nq < 2 || nq > kMaxCircuitQubits)
            return fail(Z2H_ERR_INVALID, "nq = %d outside [2, %d]", nq, kMaxCircuitQubits);
        if (dtype != Z2H_C64 && dtype != Z2H_C128) return fail(Z2H_ERR_INVALID, "unknown dtype %d", dtype);
        if (fuse < 0 || fuse > 2) return fail(Z2H_ERR_INVALID, "fuse must be 0, 1 or 2");
        if (ngates < 0 || (ngates > 0 && (!gates || !pass_of)) || !npasses) return fail(Z2H_ERR_INVALID, "arguments");
        z2h_status st = check_gates(nq, gates, ngates);
        if (st) return st;
        int limit;
        uint64_t base;
        fused_limits(nq, dtype == Z2H_C128, fuse, &limit, &base);
        if (limit == 0) {
            for (int i = 0; i < ngates; ++i) pass_of[i] = i;
            *npasses = ngates;
            return Z2H_OK;
        }
        const std::vector<std::vector<int>> plan = plan_passes(gates, ngates, limit, base);
        for (size_t p = 0; p < plan.size(); ++p)
            for (int i : plan[p]) pass_of[i] = (int32_t)p;
        *npasses = (int32_t)plan.size();
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_gates_schedule");
    }
}

z2h_status z2h_circuit_evolve(int32_t Lx, int32_t Ly, z2h_dtype dtype, void *d_state, void *d_ws, size_t ws_bytes,
                              const z2h_schedule *sched, int32_t fuse, void *stream) {
    try {
        z2h_status st = check_lattice(Lx, Ly);
        if (st) return st;
        const int nq = 2 * Lx * Ly + 1;
        if (nq > kMaxCircuitQubits) return fail(Z2H_ERR_UNSUPPORTED, "%d links plus the ancilla", nq - 1);
        if (!sched) return fail(Z2H_ERR_INVALID, "schedule is NULL");
        const z2h_schedule &S = *sched;
        if (S.steps < 0 || S.k_begin < 0 || S.k_end < S.k_begin || S.k_end > S.steps || !std::isfinite(S.dt))
            return fail(Z2H_ERR_INVALID, "schedule steps or range");
        if (S.sampling != 0 && S.sampling != 1) return fail(Z2H_ERR_INVALID, "sampling must be 0 or 1");
        if (S.order != 0 && S.order != 1) return fail(Z2H_ERR_INVALID, "order must be 0 or 1");
        for (int64_t k = S.k_begin; k < S.k_end; ++k) {
            const double s0 = S.sampling ? (double)(k + 1) / (double)S.steps : ((double)k + 0.5) / (double)S.steps;
            const double sz = S.sZ ? S.sZ[k] : s0, sx = S.sX ? S.sX[k] : s0;
            z2h_couplings cx, cz;
            const double *a = &S.start.JA, *b = &S.end.JA;
            double *px = &cx.JA, *pz = &cz.JA;
            for (int j = 0; j < 4; ++j) {
                px[j] = a[j] + sx * (b[j] - a[j]);
                pz[j] = a[j] + sz * (b[j] - a[j]);
            }
            const std::vector<z2h_gate> c = step_circuit(Lx, Ly, cx, cz, S.dt, S.order);
            if ((st = run_gates(nq, dtype, d_state, d_ws, ws_bytes, c.data(), (int)c.size(), fuse, (hipStream_t)stream)))
                return st;
        }
        return Z2H_OK;
    } catch (...) {
        return fail(Z2H_ERR_OOM, "exception in z2h_circuit_evolve");
    }
}

}  // extern "C"
