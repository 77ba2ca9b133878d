/*
 * Plain FP64 CPU state-vector oracle for the Trotterized adiabatic evolution of
 * the toric code in two transverse fields (the Z2 gauge-Higgs model in its
 * mapped form, Sec. II, Eq. (effi)).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or constant with the HIP library: it builds its own
 * lattice with its own link numbering and applies the paper's circuit factors
 * one gate at a time.  It is deliberately slow and unblocked.
 *
 * Conventions
 *   - Link numbering follows the paper's 3x3 example (Appendix, Eq. (cmt12)):
 *     horizontal links row by row, then vertical links column by column.  With
 *     h(x,y) the link from vertex (x,y) to (x+1,y) and v(x,y) the link from
 *     (x,y) to (x,y+1) on a periodic Lx x Ly lattice:
 *         h(x,y) = y*Lx + x,     v(x,y) = Lx*Ly + x*Ly + y.
 *     At 3x3 the plaquettes with lower-left corners (0,0) and (0,1) are then
 *     the paper's link sets {1,10,4,13} and {4,11,7,14} (1-based).
 *   - Bit l of a basis index is the sigma^z eigenvalue of link l: 0 <-> +1.
 *   - Rotation gates: R_a(theta) = exp(-i theta sigma^a / 2), the reading under
 *     which Eq. (gate1) holds: R_x(-g t) = exp(+i g t sigma^x / 2).
 *   - Couplings are c = (JA, JB, hx, hz):
 *       H = -JA sum_v A_v - JB sum_p B_p - hx sum_l X_l - hz sum_l Z_l.
 *     The paper's Eq. (effi) is JA = JB = 1/2, hx = g, hz = lambda.
 *
 * Every function works on an interleaved complex128 array of 2^n entries.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

/* ------------------------------------------------------------------ lattice */

/* Link index of h(x,y) (dir 0) or v(x,y) (dir 1), periodic in x and y. */
int64_t or_link(int Lx, int Ly, int x, int y, int dir)
{
    x = ((x % Lx) + Lx) % Lx;
    y = ((y % Ly) + Ly) % Ly;
    if (dir == 0)
        return (int64_t)y * Lx + x;
    return (int64_t)Lx * Ly + (int64_t)x * Ly + y;
}

/*
 * Star A_v at vertex (x,y) (Sec. II, Gauss law, Eq. (gauss)): the four links
 * touching the vertex.  Plaquette B_p with lower-left corner (x,y) (Sec. II):
 * its four sides.  Masks are stored in vertex order index = y*Lx + x.
 */
int or_masks(int Lx, int Ly, uint64_t *stars, uint64_t *plaqs)
{
    if (Lx < 2 || Ly < 2 || 2 * Lx * Ly > 62)
        return -1;
    for (int y = 0; y < Ly; y++)
        for (int x = 0; x < Lx; x++) {
            uint64_t s = 0, p = 0;
            s |= 1ull << or_link(Lx, Ly, x, y, 0);
            s |= 1ull << or_link(Lx, Ly, x - 1, y, 0);
            s |= 1ull << or_link(Lx, Ly, x, y, 1);
            s |= 1ull << or_link(Lx, Ly, x, y - 1, 1);
            p |= 1ull << or_link(Lx, Ly, x, y, 0);
            p |= 1ull << or_link(Lx, Ly, x, y + 1, 0);
            p |= 1ull << or_link(Lx, Ly, x, y, 1);
            p |= 1ull << or_link(Lx, Ly, x + 1, y, 1);
            stars[y * Lx + x] = s;
            plaqs[y * Lx + x] = p;
        }
    return 0;
}

/* Parity of the bits of i selected by mask: 0 even, 1 odd. */
static int parity(uint64_t i, uint64_t mask)
{
    return __builtin_popcountll(i & mask) & 1;
}

/* ------------------------------------------------------------ single gates */

/* Hadamard on qubit l. */
void or_h(int n, cplx *psi, int l)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t b = (int64_t)1 << l;
    const double r = 1.0 / sqrt(2.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        if (i & b)
            continue;
        cplx a = psi[i], c = psi[i | b];
        psi[i] = r * (a + c);
        psi[i | b] = r * (a - c);
    }
}

/* R_x(theta) = cos(theta/2) I - i sin(theta/2) X on qubit l. */
void or_rx(int n, cplx *psi, int l, double theta)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t b = (int64_t)1 << l;
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        if (i & b)
            continue;
        cplx a = psi[i], d = psi[i | b];
        psi[i] = c * a - I * s * d;
        psi[i | b] = c * d - I * s * a;
    }
}

/* R_z(theta) = diag(exp(-i theta/2), exp(+i theta/2)) on qubit l. */
void or_rz(int n, cplx *psi, int l, double theta)
{
    const int64_t N = (int64_t)1 << n;
    const int64_t b = (int64_t)1 << l;
    const cplx e0 = cexp(-0.5 * I * theta), e1 = cexp(0.5 * I * theta);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
        psi[i] *= (i & b) ? e1 : e0;
}

/*
 * exp(i theta Z_mask) with Z_mask the product of sigma^z over mask.  This is
 * the operator the ancilla construction of Sec. III realizes: CNOTs from the
 * masked links onto the ancilla, R_z(-2 theta) on the ancilla, CNOTs again.
 */
void or_exp_z(int n, cplx *psi, uint64_t mask, double theta)
{
    const int64_t N = (int64_t)1 << n;
    const cplx ep = cexp(I * theta), em = cexp(-I * theta);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
        psi[i] *= parity((uint64_t)i, mask) ? em : ep;
}

/*
 * exp(i theta X_mask) = cos(theta) I + i sin(theta) X_mask.  The Hadamard
 * sandwich of Sec. III (U_2) turns the Z-string version into this one.
 */
void or_exp_x(int n, cplx *psi, uint64_t mask, double theta)
{
    if (mask == 0)
        return;
    const int64_t N = (int64_t)1 << n;
    const uint64_t top = (uint64_t)1 << (63 - __builtin_clzll(mask));
    const double c = cos(theta), s = sin(theta);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        if ((uint64_t)i & top)
            continue;
        int64_t j = (int64_t)((uint64_t)i ^ mask);
        cplx a = psi[i], d = psi[j];
        psi[i] = c * a + I * s * d;
        psi[j] = c * d + I * s * a;
    }
}

/* Keep the component with even parity on mask (ancilla projected on |0>). */
static void project_even_z(int n, cplx *psi, uint64_t mask)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
        if (parity((uint64_t)i, mask))
            psi[i] = 0;
}

static double norm2(int n, const cplx *psi)
{
    const int64_t N = (int64_t)1 << n;
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < N; i++)
        s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
    return s;
}

static void scale(int n, cplx *psi, double f)
{
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
        psi[i] *= f;
}

/* ---------------------------------------------------------- initial states */

/*
 * psi_1 by the circuit of Eq. (ini1): Hadamard on every link of |0...0>, then
 * for each plaquette the parity of its four links is copied onto an ancilla
 * by CNOTs, the ancilla is projected on |0> and the CNOTs are undone.  With
 * the ancilla back in |0> the net effect on the links is to drop every basis
 * state whose plaquette parity is odd.  The result is renormalized.
 */
int or_init_psi1(int Lx, int Ly, cplx *psi)
{
    uint64_t st[64], pl[64];
    if (or_masks(Lx, Ly, st, pl))
        return -1;
    const int n = 2 * Lx * Ly;
    const int64_t N = (int64_t)1 << n;
    memset(psi, 0, sizeof(cplx) * (size_t)N);
    psi[0] = 1;
    for (int l = 0; l < n; l++)
        or_h(n, psi, l);
    for (int p = 0; p < Lx * Ly; p++)
        project_even_z(n, psi, pl[p]);
    scale(n, psi, 1.0 / sqrt(norm2(n, psi)));
    return 0;
}

/*
 * psi_1' by the circuit of Eq. (ini2): starting from |0...0>, for each star
 * the four links are rotated by Hadamards, their parity is projected even
 * through the ancilla, and the Hadamards are undone.  Renormalized.
 */
int or_init_psi1p(int Lx, int Ly, cplx *psi)
{
    uint64_t st[64], pl[64];
    if (or_masks(Lx, Ly, st, pl))
        return -1;
    const int n = 2 * Lx * Ly;
    const int64_t N = (int64_t)1 << n;
    memset(psi, 0, sizeof(cplx) * (size_t)N);
    psi[0] = 1;
    for (int v = 0; v < Lx * Ly; v++) {
        for (int l = 0; l < n; l++)
            if (st[v] >> l & 1)
                or_h(n, psi, l);
        project_even_z(n, psi, st[v]);
        for (int l = 0; l < n; l++)
            if (st[v] >> l & 1)
                or_h(n, psi, l);
    }
    scale(n, psi, 1.0 / sqrt(norm2(n, psi)));
    return 0;
}

/* ---------------------------------------------------- the Trotter step */

/*
 * exp(-i H_1 t/2) with H_1 = -hx sum_l X_l (Sec. III, Eq. (decom)): by
 * Eq. (gate1) it is prod_l R_x(-hx t).
 */
static void field_x_half(int n, cplx *psi, double hx, double t)
{
    for (int l = 0; l < n; l++)
        or_rx(n, psi, l, -hx * t);
}

/* exp(-i H_3 t) with H_3 = -hz sum_l Z_l: prod_l R_z(-2 hz t) (Eq. (gate1)). */
static void field_z_full(int n, cplx *psi, double hz, double t)
{
    for (int l = 0; l < n; l++)
        or_rz(n, psi, l, -2.0 * hz * t);
}

/*
 * exp(-i H_2 t/2) with H_2 = -JA sum_v A_v - JB sum_p B_p (Eq. (decom)):
 * prod_v exp(i JA A_v t/2) prod_p exp(i JB B_p t/2); the plaquette factors
 * act first (right to left, Sec. III).
 */
static void stabilizer_half(int n, cplx *psi, int nv, const uint64_t *st,
                            const uint64_t *pl, double JA, double JB, double t)
{
    for (int p = 0; p < nv; p++)
        or_exp_z(n, psi, pl[p], JB * t / 2);
    for (int v = 0; v < nv; v++)
        or_exp_x(n, psi, st[v], JA * t / 2);
}

/*
 * One second-order Trotter-Suzuki step of Sec. III:
 *   exp(-iH t) ~ exp(-iH_1 t/2) exp(-iH_2 t/2) exp(-iH_3 t) exp(-iH_2 t/2) exp(-iH_1 t/2)
 * applied right to left.  cx = couplings used by the sigma^x-type terms
 * (JA, hx: entries 0 and 2 of cx), cz = couplings used by the sigma^z-type
 * terms (JB, hz: entries 1 and 3 of cz); in the plain method both are the
 * couplings at the step's parameter value.
 *
 * order = 1 swaps the roles of H_1 and H_3 (outer halves are the z field),
 * a variant used only by the self-duality check of Sec. III.
 */
void or_trotter_step(int Lx, int Ly, cplx *psi, const double *cx,
                     const double *cz, double t, int order)
{
    uint64_t st[64], pl[64];
    or_masks(Lx, Ly, st, pl);
    const int n = 2 * Lx * Ly, nv = Lx * Ly;
    const double JA = cx[0], hx = cx[2], JB = cz[1], hz = cz[3];
    if (order == 0) {
        field_x_half(n, psi, hx, t);
        stabilizer_half(n, psi, nv, st, pl, JA, JB, t);
        field_z_full(n, psi, hz, t);
        stabilizer_half(n, psi, nv, st, pl, JA, JB, t);
        field_x_half(n, psi, hx, t);
    } else {
        /* exp(-iH_3 t/2) exp(-iH_2 t/2) exp(-iH_1 t) exp(-iH_2 t/2) exp(-iH_3 t/2) */
        field_z_full(n, psi, hz, t / 2);
        stabilizer_half(n, psi, nv, st, pl, JA, JB, t);
        field_x_half(n, psi, hx, 2 * t);
        stabilizer_half(n, psi, nv, st, pl, JA, JB, t);
        field_z_full(n, psi, hz, t / 2);
    }
}

/*
 * The adiabatic ramp of Sec. III: M steps of equal duration dt, the
 * couplings moving on the straight line c(s) = (1-s) c0 + s c1.  The
 * parameter value used inside step k (0-based) is
 *     sampling 0: s_k = (k + 1/2)/M   (midpoint)
 *     sampling 1: s_k = (k + 1)/M     (right end, g = k*dg of the Appendix)
 * unless per-step values are passed: sZ[k] drives the z-type couplings
 * (JB, hz) and sX[k] the x-type couplings (JA, hx) of step k.
 */
int or_evolve(int Lx, int Ly, cplx *psi, const double *c0, const double *c1,
              int64_t M, double dt, const double *sZ, const double *sX,
              int sampling, int order)
{
    if (Lx < 2 || Ly < 2 || 2 * Lx * Ly > 40 || M < 0)
        return -1;
    for (int64_t k = 0; k < M; k++) {
        double s = sampling ? (double)(k + 1) / (double)M
                            : ((double)k + 0.5) / (double)M;
        double szk = sZ ? sZ[k] : s, sxk = sX ? sX[k] : s;
        double cx[4], cz[4];
        for (int a = 0; a < 4; a++) {
            cx[a] = (1 - sxk) * c0[a] + sxk * c1[a];
            cz[a] = (1 - szk) * c0[a] + szk * c1[a];
        }
        or_trotter_step(Lx, Ly, psi, cx, cz, dt, order);
    }
    return 0;
}

/* ------------------------------------------------------------ observables */

/* <Z_mask> = sum_i |psi_i|^2 (-1)^{parity(i & mask)} */
double or_expect_z(int n, const cplx *psi, uint64_t mask)
{
    const int64_t N = (int64_t)1 << n;
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < N; i++) {
        double p = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
        s += parity((uint64_t)i, mask) ? -p : p;
    }
    return s;
}

/* <X_mask> = Re sum_i conj(psi_i) psi_{i xor mask} */
double or_expect_x(int n, const cplx *psi, uint64_t mask)
{
    const int64_t N = (int64_t)1 << n;
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < N; i++)
        s += creal(conj(psi[i]) * psi[(uint64_t)i ^ mask]);
    return s;
}

/*
 * out[0] = <psi|psi>, out[1] = <H(c)>, out[2] = sum_v <A_v>,
 * out[3] = sum_p <B_p>, out[4] = mean_l <X_l>, out[5] = mean_l <Z_l>.
 * Expectations are unnormalized sums (divide by out[0] for a non-unit norm).
 */
int or_observe(int Lx, int Ly, const cplx *psi, const double *c, double *out)
{
    uint64_t st[64], pl[64];
    if (or_masks(Lx, Ly, st, pl))
        return -1;
    const int n = 2 * Lx * Ly, nv = Lx * Ly;
    double sa = 0, sb = 0, sx = 0, sz = 0;
    for (int v = 0; v < nv; v++) {
        sa += or_expect_x(n, psi, st[v]);
        sb += or_expect_z(n, psi, pl[v]);
    }
    for (int l = 0; l < n; l++) {
        sx += or_expect_x(n, psi, (uint64_t)1 << l);
        sz += or_expect_z(n, psi, (uint64_t)1 << l);
    }
    out[0] = norm2(n, psi);
    out[1] = -c[0] * sa - c[1] * sb - c[2] * sx - c[3] * sz;
    out[2] = sa;
    out[3] = sb;
    out[4] = sx / n;
    out[5] = sz / n;
    return 0;
}

/*
 * Distribution of |psi|^2 over the eigenvalues of Ztilde = -sum_l Z_l
 * (Sec. V): out[w] = sum of |psi_i|^2 over basis states with w links in
 * sigma^z = -1, i.e. Ztilde = 2w - n.
 */
void or_weight_hist(int n, const cplx *psi, double *out)
{
    const int64_t N = (int64_t)1 << n;
    for (int w = 0; w <= n; w++)
        out[w] = 0;
    for (int64_t i = 0; i < N; i++)
        out[__builtin_popcountll((uint64_t)i)] +=
            creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
}
