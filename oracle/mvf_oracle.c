/*
 * mvf_oracle.c -- plain, slow CPU oracle for subdomain Mean-Value-Form bounding.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * GPU library.
 *
 * What it computes (arXiv 2507.20769):
 *   - outward-rounded interval arithmetic (Sec. 2.2, "Interval Arithmetic";
 *     Sec. 3.2 on directed rounding for + - * / sqrt and double-direction
 *     padding for the other intrinsics);
 *   - the Natural Interval Extension of a factorable function given as a DAG
 *     (Sec. 2.2, definition "Factorable function" and the paragraph after it;
 *     Sec. 3.2, Fig. "DAG_NIE");
 *   - tangent-mode interval derivatives (Sec. 3.2, tangent structure) and a
 *     reverse-mode interval adjoint of the same DAG;
 *   - the Mean Value Form f(m(X)) + <grad F(X), X - m(X)> (Sec. 2.2,
 *     Definition "Mean Value Form"), intersected with the natural extension;
 *   - uniform splitting of a box into subdomains, dimension 1 fastest
 *     (Sec. 2.2 splitting technique, step i; Sec. 3.1.1 worked example);
 *   - the refinement = interval hull over subdomains (Sec. 2.2 splitting
 *     technique, step iii; Sec. 3.1 Step 3), with the objective argmin.
 *
 * Every rounded operation sets the FPU rounding mode explicitly around one
 * scalar operation (fesetround), so each result is the correctly rounded
 * value in the stated direction.  Build with -frounding-math
 * -ffp-contract=off -fno-fast-math on x86-64 (SSE2 double arithmetic).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   * breakpoints   b_{i,0}=lo_i, b_{i,s}=hi_i,
 *                   b_{i,j}=min(hi_i, RN(lo_i + RN(j*h_i))), h_i=RN(RN(hi_i-lo_i)/s_i);
 *   * centre        c_i = RN(0.5*RN(b_lo+b_hi));
 *   * f(m(X))       evaluated as an interval at degenerate [c_i,c_i];
 *   * exp/log       libm result in round-to-nearest, widened by two ulps on
 *                   each side (exp lower end clamped at 0);
 *   * tanh/sin/cos  libm result in round-to-nearest widened by four ulps on
 *                   each side, clamped to [-1, 1]; sin and cos take +-1 where
 *                   the argument interval may contain an extremum (the
 *                   interval (X - c) / [2pi] contains an integer, in outward
 *                   rounding with pi enclosed by two doubles), and are
 *                   [-1, 1] when RU(hi - lo) >= 6.28;
 *   * derivatives   the tangent and adjoint rules written next to each op
 *                   below (each is an interval inclusion of the true
 *                   derivative); division by V uses the reciprocal interval
 *                   1/V = [RD(1/d), RU(1/c)];
 *   * domain        0 in a divisor, a negative sqrt argument, a
 *                   non-positive log argument, or a NaN in any final bound
 *                   flags the subdomain and sets all its bounds to [-inf,+inf];
 *   * MVF inner product accumulated for i = 1..n starting from [f(c)].
 */
#define _GNU_SOURCE
#include <fenv.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#pragma STDC FENV_ACCESS ON

enum { OP_VAR = 0, OP_CONST, OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_SQR, OP_SQRT, OP_EXP, OP_LOG, OP_TANH, OP_SIN,
       OP_COS };
enum { MODE_NIE = 0, MODE_MVF = 1, MODE_BOTH = 2 };
enum { GRAD_FWD = 0, GRAD_REV = 1 };
/* root kinds: the objective or an unconstrained function, g <= 0, h = 0 (Sec. 3.1, the NLP) */
enum { ORC_FREE = 0, ORC_INEQ = 1, ORC_EQ = 2 };

typedef struct { int32_t op, a, b; } orc_node;
typedef struct { double lo, hi; } ivl;

/* ------------------------------------------------------------------------ */
/* directed rounding of single operations                                   */
/* ------------------------------------------------------------------------ */

#define BARRIER(x) __asm__ volatile("" : "+x"(x))

static double rnd_add(int mode, double a, double b) {
    fesetround(mode); BARRIER(a); BARRIER(b);
    double r = a + b; BARRIER(r);
    fesetround(FE_TONEAREST);
    return r;
}
static double rnd_sub(int mode, double a, double b) {
    fesetround(mode); BARRIER(a); BARRIER(b);
    double r = a - b; BARRIER(r);
    fesetround(FE_TONEAREST);
    return r;
}
static double rnd_mul(int mode, double a, double b) {
    fesetround(mode); BARRIER(a); BARRIER(b);
    double r = a * b; BARRIER(r);
    fesetround(FE_TONEAREST);
    return r;
}
static double rnd_div(int mode, double a, double b) {
    fesetround(mode); BARRIER(a); BARRIER(b);
    double r = a / b; BARRIER(r);
    fesetround(FE_TONEAREST);
    return r;
}
static double rnd_sqrt(int mode, double a) {
    fesetround(mode); BARRIER(a);
    double r = sqrt(a); BARRIER(r);
    fesetround(FE_TONEAREST);
    return r;
}
#define RD FE_DOWNWARD
#define RU FE_UPWARD

static double dn2(double x) { return nextafter(nextafter(x, -INFINITY), -INFINITY); }
static double up2(double x) { return nextafter(nextafter(x, INFINITY), INFINITY); }

/* exported for the rounding pins */
double orc_round_op(int op, int dir, double a, double b) {
    int mode = dir < 0 ? RD : (dir > 0 ? RU : FE_TONEAREST);
    switch (op) {
    case OP_ADD: return rnd_add(mode, a, b);
    case OP_SUB: return rnd_sub(mode, a, b);
    case OP_MUL: return rnd_mul(mode, a, b);
    case OP_DIV: return rnd_div(mode, a, b);
    case OP_SQRT: return rnd_sqrt(mode, a);
    default: return NAN;
    }
}

/* ------------------------------------------------------------------------ */
/* interval operations                                                      */
/* ------------------------------------------------------------------------ */

static ivl I(double lo, double hi) { ivl r = {lo, hi}; return r; }

static ivl iadd(ivl u, ivl v) { return I(rnd_add(RD, u.lo, v.lo), rnd_add(RU, u.hi, v.hi)); }
static ivl isub(ivl u, ivl v) { return I(rnd_sub(RD, u.lo, v.hi), rnd_sub(RU, u.hi, v.lo)); }

/* [a,b]*[c,d]: hull of the four endpoint products, each rounded outward. */
static ivl imul(ivl u, ivl v) {
    double p[4] = {u.lo, u.lo, u.hi, u.hi}, q[4] = {v.lo, v.hi, v.lo, v.hi};
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < 4; ++i) {
        lo = fmin(lo, rnd_mul(RD, p[i], q[i]));
        hi = fmax(hi, rnd_mul(RU, p[i], q[i]));
    }
    return I(lo, hi);
}

/* [a,b]/[c,d] with 0 not in [c,d]: hull of the four endpoint quotients. */
static ivl idiv(ivl u, ivl v) {
    double p[4] = {u.lo, u.lo, u.hi, u.hi}, q[4] = {v.lo, v.hi, v.lo, v.hi};
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < 4; ++i) {
        lo = fmin(lo, rnd_div(RD, p[i], q[i]));
        hi = fmax(hi, rnd_div(RU, p[i], q[i]));
    }
    return I(lo, hi);
}

/* 1/[c,d] with 0 not in [c,d] */
static ivl irecip(ivl v) { return I(rnd_div(RD, 1.0, v.hi), rnd_div(RU, 1.0, v.lo)); }

static ivl isqr(ivl u) {
    if (u.lo >= 0) return I(rnd_mul(RD, u.lo, u.lo), rnd_mul(RU, u.hi, u.hi));
    if (u.hi <= 0) return I(rnd_mul(RD, u.hi, u.hi), rnd_mul(RU, u.lo, u.lo));
    return I(0.0, fmax(rnd_mul(RU, u.lo, u.lo), rnd_mul(RU, u.hi, u.hi)));
}

static ivl isqrt(ivl u) { return I(rnd_sqrt(RD, u.lo), rnd_sqrt(RU, u.hi)); }

static ivl iexp(ivl u) { return I(fmax(0.0, dn2(exp(u.lo))), up2(exp(u.hi))); }
static ivl ilog(ivl u) { return I(dn2(log(u.lo)), up2(log(u.hi))); }

static double dn4(double x) { return dn2(dn2(x)); }
static double up4(double x) { return up2(up2(x)); }

/* tanh is increasing with values in (-1, 1) */
static ivl itanh(ivl u) { return I(fmax(-1.0, dn4(tanh(u.lo))), fmin(1.0, up4(tanh(u.hi)))); }

/* pi lies between these neighbouring doubles */
#define PI_LO 3.141592653589793
#define PI_HI 3.1415926535897936

/* can X contain c + 2 k pi for an integer k?  T = (X - C) / [2 pi] in outward
 * rounding; true when T contains an integer or is not finite */
static int may_contain(ivl x, ivl c) {
    ivl t = idiv(isub(x, c), I(2.0 * PI_LO, 2.0 * PI_HI));
    if (!isfinite(t.lo) || !isfinite(t.hi)) return 1;
    return ceil(t.lo) <= t.hi;
}

/* sin over [a, b]: the endpoint values, and +-1 where an extremum may lie
 * inside; the whole range [-1, 1] from width 6.28 on */
static ivl isin(ivl u) {
    double sa = sin(u.lo), sb = sin(u.hi);
    double lo = fmin(dn4(sa), dn4(sb)), hi = fmax(up4(sa), up4(sb));
    if (may_contain(u, I(PI_LO / 2, PI_HI / 2))) hi = 1.0;          /* pi/2 + 2 k pi */
    if (may_contain(u, I(-PI_HI / 2, -PI_LO / 2))) lo = -1.0;       /* -pi/2 + 2 k pi */
    if (!(rnd_sub(RU, u.hi, u.lo) < 6.28)) { lo = -1.0; hi = 1.0; }
    return I(fmax(-1.0, lo), fmin(1.0, hi));
}
/* cos: maxima at 2 k pi, minima at pi + 2 k pi */
static ivl icos(ivl u) {
    double ca = cos(u.lo), cb = cos(u.hi);
    double lo = fmin(dn4(ca), dn4(cb)), hi = fmax(up4(ca), up4(cb));
    if (may_contain(u, I(0.0, 0.0))) hi = 1.0;
    if (may_contain(u, I(PI_LO, PI_HI))) lo = -1.0;
    if (!(rnd_sub(RU, u.hi, u.lo) < 6.28)) { lo = -1.0; hi = 1.0; }
    return I(fmax(-1.0, lo), fmin(1.0, hi));
}
static ivl ineg(ivl u) { return I(-u.hi, -u.lo); }

/* 2*U, exact up to overflow */
static ivl itwice(ivl u) { return I(rnd_add(RD, u.lo, u.lo), rnd_add(RU, u.hi, u.hi)); }

/* enclosure of 1/(2*sqrt(u)) given Z = sqrt(U): 1/[2z_lo, 2z_hi], with an
 * unbounded upper end when z_lo is zero */
static ivl isqrt_deriv(ivl z) {
    ivl t = itwice(z);
    if (t.lo <= 0) return I(rnd_div(RD, 1.0, t.hi), INFINITY);
    return irecip(t);
}

/* exported for the hand-worked interval pins */
void orc_interval_op(int op, const double *u, const double *v, double *z) {
    ivl U = I(u[0], u[1]), V = v ? I(v[0], v[1]) : I(0, 0), Z;
    switch (op) {
    case OP_ADD: Z = iadd(U, V); break;
    case OP_SUB: Z = isub(U, V); break;
    case OP_MUL: Z = imul(U, V); break;
    case OP_DIV: Z = idiv(U, V); break;
    case OP_SQR: Z = isqr(U); break;
    case OP_SQRT: Z = isqrt(U); break;
    case OP_EXP: Z = iexp(U); break;
    case OP_LOG: Z = ilog(U); break;
    case OP_TANH: Z = itanh(U); break;
    case OP_SIN: Z = isin(U); break;
    case OP_COS: Z = icos(U); break;
    default: Z = I(NAN, NAN);
    }
    z[0] = Z.lo; z[1] = Z.hi;
}

/* ------------------------------------------------------------------------ */
/* tape evaluation                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_node *nodes;
    int32_t n_nodes;
    const double *consts;
    int32_t n_vars;
    const int32_t *roots;
    int32_t n_roots;
    uint8_t *live;      /* node reachable from some root */
    uint8_t *cone;      /* [n_roots][n_nodes] node reachable from root r */
} orc_tape;

static void tape_init(orc_tape *t, const orc_node *nodes, int32_t n_nodes, const double *consts, int32_t n_vars,
                      const int32_t *roots, int32_t n_roots) {
    t->nodes = nodes; t->n_nodes = n_nodes; t->consts = consts; t->n_vars = n_vars;
    t->roots = roots; t->n_roots = n_roots;
    t->live = calloc((size_t)n_nodes + 1, 1);
    t->cone = calloc((size_t)n_nodes * n_roots + 1, 1);
    for (int r = 0; r < n_roots; ++r) {
        uint8_t *c = t->cone + (size_t)r * n_nodes;
        c[roots[r]] = 1;
        for (int i = n_nodes - 1; i >= 0; --i) {
            if (!c[i]) continue;
            t->live[i] = 1;
            int op = nodes[i].op;
            if (op >= OP_ADD) c[nodes[i].a] = 1;
            if (op >= OP_ADD && op <= OP_DIV) c[nodes[i].b] = 1;
        }
    }
}
static void tape_free(orc_tape *t) { free(t->live); free(t->cone); }

/* Natural interval extension of every live node on box X (NIE).  Returns
 * nonzero on a domain violation. */
static int eval_values(const orc_tape *t, const ivl *X, ivl *val) {
    int bad = 0;
    for (int i = 0; i < t->n_nodes; ++i) {
        if (!t->live[i]) { val[i] = I(0, 0); continue; }
        const orc_node *nd = &t->nodes[i];
        ivl U = nd->op >= OP_ADD ? val[nd->a] : I(0, 0);
        ivl V = (nd->op >= OP_ADD && nd->op <= OP_DIV) ? val[nd->b] : I(0, 0);
        switch (nd->op) {
        case OP_VAR: val[i] = X[nd->a]; break;
        case OP_CONST: val[i] = I(t->consts[nd->a], t->consts[nd->a]); break;
        case OP_ADD: val[i] = iadd(U, V); break;
        case OP_SUB: val[i] = isub(U, V); break;
        case OP_MUL: val[i] = imul(U, V); break;
        case OP_DIV:
            if (V.lo <= 0 && V.hi >= 0) { bad = 1; val[i] = I(-INFINITY, INFINITY); }
            else val[i] = idiv(U, V);
            break;
        case OP_SQR: val[i] = isqr(U); break;
        case OP_SQRT:
            if (U.lo < 0) { bad = 1; val[i] = I(-INFINITY, INFINITY); }
            else val[i] = isqrt(U);
            break;
        case OP_EXP: val[i] = iexp(U); break;
        case OP_LOG:
            if (U.lo <= 0) { bad = 1; val[i] = I(-INFINITY, INFINITY); }
            else val[i] = ilog(U);
            break;
        case OP_TANH: val[i] = itanh(U); break;
        case OP_SIN: val[i] = isin(U); break;
        case OP_COS: val[i] = icos(U); break;
        default: bad = 1;
        }
    }
    return bad;
}

/* Tangent mode: val as above, plus tan[i*n + j] = d node_i / d x_j. */
static int eval_tangents(const orc_tape *t, const ivl *X, ivl *val, ivl *tan) {
    const int n = t->n_vars;
    int bad = eval_values(t, X, val);
    if (bad) return bad;
    for (int i = 0; i < t->n_nodes; ++i) {
        ivl *dz = tan + (size_t)i * n;
        if (!t->live[i]) { for (int j = 0; j < n; ++j) dz[j] = I(0, 0); continue; }
        const orc_node *nd = &t->nodes[i];
        const ivl *du = nd->op >= OP_ADD ? tan + (size_t)nd->a * n : NULL;
        const ivl *dv = (nd->op >= OP_ADD && nd->op <= OP_DIV) ? tan + (size_t)nd->b * n : NULL;
        ivl U = nd->op >= OP_ADD ? val[nd->a] : I(0, 0);
        ivl V = (nd->op >= OP_ADD && nd->op <= OP_DIV) ? val[nd->b] : I(0, 0);
        ivl Z = val[i], R;
        switch (nd->op) {
        case OP_VAR:   /* e_i */
            for (int j = 0; j < n; ++j) dz[j] = j == nd->a ? I(1, 1) : I(0, 0);
            break;
        case OP_CONST:
            for (int j = 0; j < n; ++j) dz[j] = I(0, 0);
            break;
        case OP_ADD:   /* dU + dV */
            for (int j = 0; j < n; ++j) dz[j] = iadd(du[j], dv[j]);
            break;
        case OP_SUB:   /* dU - dV */
            for (int j = 0; j < n; ++j) dz[j] = isub(du[j], dv[j]);
            break;
        case OP_MUL:   /* V*dU + U*dV */
            for (int j = 0; j < n; ++j) dz[j] = iadd(imul(V, du[j]), imul(U, dv[j]));
            break;
        case OP_DIV:   /* (dU - Z*dV) * (1/V) */
            R = irecip(V);
            for (int j = 0; j < n; ++j) dz[j] = imul(isub(du[j], imul(Z, dv[j])), R);
            break;
        case OP_SQR:   /* (2U) * dU */
            R = itwice(U);
            for (int j = 0; j < n; ++j) dz[j] = imul(R, du[j]);
            break;
        case OP_SQRT:  /* dU * 1/(2Z) */
            R = isqrt_deriv(Z);
            for (int j = 0; j < n; ++j) dz[j] = imul(du[j], R);
            break;
        case OP_EXP:   /* Z * dU */
            for (int j = 0; j < n; ++j) dz[j] = imul(Z, du[j]);
            break;
        case OP_LOG:   /* dU * (1/U) */
            R = irecip(U);
            for (int j = 0; j < n; ++j) dz[j] = imul(du[j], R);
            break;
        case OP_TANH:  /* (1 - Z^2) * dU */
            R = isub(I(1, 1), isqr(Z));
            for (int j = 0; j < n; ++j) dz[j] = imul(R, du[j]);
            break;
        case OP_SIN:   /* cos(U) * dU */
            R = icos(U);
            for (int j = 0; j < n; ++j) dz[j] = imul(R, du[j]);
            break;
        case OP_COS:   /* -sin(U) * dU */
            R = ineg(isin(U));
            for (int j = 0; j < n; ++j) dz[j] = imul(R, du[j]);
            break;
        }
    }
    return 0;
}

/* Reverse sweep over the nodes with nonzero cone mask, in descending index,
 * starting from adjoints adj[] (already seeded).  A contribution to a
 * variable leaf goes straight into that variable's gradient accumulator G[]
 * (in sweep order); contributions to constants are dropped.  val holds the
 * values from eval_values. */
static void acc_to(const orc_tape *t, int x, ivl c, ivl *adj, ivl *G) {
    const orc_node *nd = &t->nodes[x];
    if (nd->op == OP_VAR) G[nd->a] = iadd(G[nd->a], c);
    else if (nd->op != OP_CONST) adj[x] = iadd(adj[x], c);
}
static void sub_from(const orc_tape *t, int x, ivl c, ivl *adj, ivl *G) {
    const orc_node *nd = &t->nodes[x];
    if (nd->op == OP_VAR) G[nd->a] = isub(G[nd->a], c);
    else if (nd->op != OP_CONST) adj[x] = isub(adj[x], c);
}

static void reverse_sweep(const orc_tape *t, const uint8_t *mask, const ivl *val, ivl *adj, ivl *G) {
    for (int i = t->n_nodes - 1; i >= 0; --i) {
        if (!mask[i]) continue;
        const orc_node *nd = &t->nodes[i];
        ivl zb = adj[i], T;
        switch (nd->op) {
        case OP_VAR: case OP_CONST: break;        /* handled by the consumers */
        case OP_ADD:   /* ub += zb; vb += zb */
            acc_to(t, nd->a, zb, adj, G);
            acc_to(t, nd->b, zb, adj, G);
            break;
        case OP_SUB:   /* ub += zb; vb -= zb */
            acc_to(t, nd->a, zb, adj, G);
            sub_from(t, nd->b, zb, adj, G);
            break;
        case OP_MUL:   /* ub += zb*V; vb += zb*U */
            acc_to(t, nd->a, imul(zb, val[nd->b]), adj, G);
            acc_to(t, nd->b, imul(zb, val[nd->a]), adj, G);
            break;
        case OP_DIV:   /* t = zb*(1/V); ub += t; vb -= t*Z */
            T = imul(zb, irecip(val[nd->b]));
            acc_to(t, nd->a, T, adj, G);
            sub_from(t, nd->b, imul(T, val[i]), adj, G);
            break;
        case OP_SQR:   /* ub += zb*(2U) */
            acc_to(t, nd->a, imul(zb, itwice(val[nd->a])), adj, G);
            break;
        case OP_SQRT:  /* ub += zb*1/(2Z) */
            acc_to(t, nd->a, imul(zb, isqrt_deriv(val[i])), adj, G);
            break;
        case OP_EXP:   /* ub += zb*Z */
            acc_to(t, nd->a, imul(zb, val[i]), adj, G);
            break;
        case OP_LOG:   /* ub += zb*(1/U) */
            acc_to(t, nd->a, imul(zb, irecip(val[nd->a])), adj, G);
            break;
        case OP_TANH:  /* ub += zb*(1 - Z^2) */
            acc_to(t, nd->a, imul(zb, isub(I(1, 1), isqr(val[i]))), adj, G);
            break;
        case OP_SIN:   /* ub += zb*cos(U) */
            acc_to(t, nd->a, imul(zb, icos(val[nd->a])), adj, G);
            break;
        case OP_COS:   /* ub += zb*(-sin(U)) */
            acc_to(t, nd->a, imul(zb, ineg(isin(val[nd->a]))), adj, G);
            break;
        }
    }
}

/* interval gradient of root r on box X; returns nonzero on domain violation */
static int gradient_rev(const orc_tape *t, int r, const ivl *val, ivl *adj, ivl *G) {
    for (int i = 0; i < t->n_nodes; ++i) adj[i] = I(0, 0);
    for (int j = 0; j < t->n_vars; ++j) G[j] = I(0, 0);
    acc_to(t, t->roots[r], I(1, 1), adj, G);
    reverse_sweep(t, t->cone + (size_t)r * t->n_nodes, val, adj, G);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* splitting (Step 1)                                                       */
/* ------------------------------------------------------------------------ */

static double breakpoint(double lo, double hi, int32_t s, int64_t j) {
    if (j <= 0) return lo;
    if (j >= s) return hi;
    double w = hi - lo;                 /* round to nearest */
    double h = w / (double)s;
    double r = lo + (double)j * h;
    return fmin(hi, r);
}

/* subdomain k of box [n][2] split by s[n], dimension 0 fastest */
static void subdomain(int n, const double *box, const int32_t *s, int64_t k, ivl *X, double *c) {
    for (int i = 0; i < n; ++i) {
        int64_t j = k % s[i];
        k /= s[i];
        double lo = breakpoint(box[2 * i], box[2 * i + 1], s[i], j);
        double hi = breakpoint(box[2 * i], box[2 * i + 1], s[i], j + 1);
        X[i] = I(lo, hi);
        c[i] = 0.5 * (lo + hi);
    }
}

void orc_subdomain(int n, const double *box, const int32_t *s, int64_t k, double *X, double *c) {
    ivl Xi[256];
    subdomain(n, box, s, k, Xi, c);
    for (int i = 0; i < n; ++i) { X[2 * i] = Xi[i].lo; X[2 * i + 1] = Xi[i].hi; }
}

/* ------------------------------------------------------------------------ */
/* one subdomain: NIE, point pass, gradient, MVF combine (Step 2)           */
/* ------------------------------------------------------------------------ */

typedef struct {
    orc_tape *t;
    int mode, grad;
    ivl *val, *pval, *tan, *adj, *G;
} orc_ws;

static void ws_alloc(orc_ws *w, orc_tape *t, int mode, int grad) {
    size_t N = (size_t)t->n_nodes + 1, n = (size_t)t->n_vars + 1;
    w->t = t; w->mode = mode; w->grad = grad;
    w->val = malloc(N * sizeof(ivl));
    w->pval = malloc(N * sizeof(ivl));
    w->adj = malloc(N * sizeof(ivl));
    w->G = malloc(n * t->n_roots * sizeof(ivl) + sizeof(ivl));
    w->tan = grad == GRAD_FWD && mode != MODE_NIE ? malloc(N * n * sizeof(ivl)) : NULL;
}
static void ws_free(orc_ws *w) { free(w->val); free(w->pval); free(w->adj); free(w->G); free(w->tan); }

/* bounds B[r] of every root on box X with centre c; returns the flag */
static uint32_t bound_one(orc_ws *w, const ivl *X, const double *c, ivl *B) {
    orc_tape *t = w->t;
    const int n = t->n_vars, m = t->n_roots;
    int bad;
    if (w->mode == MODE_NIE) {
        bad = eval_values(t, X, w->val);
    } else if (w->grad == GRAD_FWD) {
        bad = eval_tangents(t, X, w->val, w->tan);
    } else {
        bad = eval_values(t, X, w->val);
    }
    ivl Cp[256];
    for (int i = 0; i < n; ++i) Cp[i] = I(c[i], c[i]);
    if (!bad && w->mode != MODE_NIE) bad = eval_values(t, Cp, w->pval);
    uint32_t flag = bad ? 1u : 0u;
    for (int r = 0; r < m && !bad; ++r) {
        ivl nie = w->val[t->roots[r]];
        if (w->mode == MODE_NIE) { B[r] = nie; continue; }
        ivl *G = w->G + (size_t)r * n;
        if (w->grad == GRAD_FWD) {
            for (int j = 0; j < n; ++j) G[j] = w->tan[(size_t)t->roots[r] * n + j];
        } else {
            gradient_rev(t, r, w->val, w->adj, G);
        }
        ivl acc = w->pval[t->roots[r]];
        for (int i = 0; i < n; ++i) {
            ivl D = I(rnd_sub(RD, X[i].lo, c[i]), rnd_sub(RU, X[i].hi, c[i]));
            acc = iadd(acc, imul(G[i], D));
        }
        if (w->mode == MODE_MVF) B[r] = acc;
        else B[r] = I(fmax(acc.lo, nie.lo), fmin(acc.hi, nie.hi));
    }
    for (int r = 0; r < m && !flag; ++r)
        if (isnan(B[r].lo) || isnan(B[r].hi)) flag = 1;
    if (flag)
        for (int r = 0; r < m; ++r) B[r] = I(-INFINITY, INFINITY);
    return flag;
}

/* ------------------------------------------------------------------------ */
/* exported: bound a box (Steps 1-3)                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    orc_tape *t;
    const double *box;
    const int32_t *splits;
    const int64_t *ks;          /* explicit subdomain list, or NULL */
    int64_t k0, k1, kbase;      /* this job's range; kbase = first index of the call */
    int mode, grad;
    const int32_t *kinds;       /* [m] root kinds (ORC_FREE / ORC_INEQ / ORC_EQ) or NULL */
    double *per_sub;            /* [m][2][count] or NULL */
    uint32_t *flags;            /* [count] or NULL */
    int64_t count;
    double *red;                /* [m][2] */
    int64_t argmin;
    double filtered_lo, ub;     /* feasibility-filtered objective bound; upper bound from centres */
} orc_job;

/*
 * Subdomain k is proven infeasible when a constraint's bound excludes it: an
 * inequality g <= 0 with lower bound > 0, an equality h = 0 whose bound does
 * not contain 0 (the feasibility check of Sec. 3.1 applied per subdomain).
 */
static int proven_infeasible(const int32_t *kinds, int m, const ivl *B) {
    if (!kinds) return 0;
    for (int r = 1; r < m; ++r) {
        if (kinds[r] == ORC_INEQ && B[r].lo > 0) return 1;
        if (kinds[r] == ORC_EQ && (B[r].lo > 0 || B[r].hi < 0)) return 1;
    }
    return 0;
}

/*
 * The centre c_k is a rigorously feasible point when every inequality's
 * enclosure at c_k has upper bound <= 0 (no equality constraints: a point
 * cannot be shown to satisfy h = 0); then hi(f(c_k)) bounds the minimum from
 * above.  Needs the point pass (MVF modes) and an unflagged subdomain.
 */
static double centre_upper_bound(const orc_tape *t, const int32_t *kinds, const ivl *pval) {
    const int m = t->n_roots;
    for (int r = 1; r < m && kinds; ++r) {
        if (kinds[r] == ORC_EQ) return INFINITY;
        if (kinds[r] == ORC_INEQ && !(pval[t->roots[r]].hi <= 0)) return INFINITY;
    }
    return pval[t->roots[0]].hi;
}

static void *bound_range(void *arg) {
    orc_job *jb = arg;
    orc_tape *t = jb->t;
    const int n = t->n_vars, m = t->n_roots;
    orc_ws w;
    ws_alloc(&w, t, jb->mode, jb->grad);
    ivl X[256], B[64];
    double c[256];
    for (int r = 0; r < m; ++r) { jb->red[2 * r] = INFINITY; jb->red[2 * r + 1] = -INFINITY; }
    jb->argmin = -1;
    jb->filtered_lo = INFINITY;
    jb->ub = INFINITY;
    for (int64_t q = jb->k0; q < jb->k1; ++q) {
        int64_t k = jb->ks ? jb->ks[q] : q;
        subdomain(n, jb->box, jb->splits, k, X, c);
        uint32_t f = bound_one(&w, X, c, B);
        int64_t o = q - jb->kbase;
        if (jb->flags) jb->flags[o] = f;
        if (!proven_infeasible(jb->kinds, m, B)) jb->filtered_lo = fmin(jb->filtered_lo, B[0].lo);
        if (!f && jb->mode != MODE_NIE) jb->ub = fmin(jb->ub, centre_upper_bound(t, jb->kinds, w.pval));
        for (int r = 0; r < m; ++r) {
            if (jb->per_sub) {
                jb->per_sub[((size_t)r * 2 + 0) * jb->count + o] = B[r].lo;
                jb->per_sub[((size_t)r * 2 + 1) * jb->count + o] = B[r].hi;
            }
            if (r == 0 && (B[0].lo < jb->red[0] || jb->argmin < 0)) jb->argmin = k;
            jb->red[2 * r] = fmin(jb->red[2 * r], B[r].lo);
            jb->red[2 * r + 1] = fmax(jb->red[2 * r + 1], B[r].hi);
        }
    }
    ws_free(&w);
    return NULL;
}

/*
 * Bound the subdomains k in [k0, k1) of box (or the explicit list ks[k0..k1)
 * when ks != NULL; the list must be ascending for the argmin tie rule).  per_sub[m][2][k1-k0] (nullable), flags[k1-k0] (nullable),
 * reduced[m][2], argmin (smallest k attaining the objective lower bound).
 * Work is split over nthreads contiguous ranges.  Returns 0.
 */
int orc_bound(const orc_node *nodes, int32_t n_nodes, const double *consts, int32_t n_vars,
              const int32_t *roots, int32_t n_roots, const double *box, const int32_t *splits,
              const int64_t *ks, int64_t k0, int64_t k1, int mode, int grad, const int32_t *kinds,
              double *per_sub, uint32_t *flags, double *reduced, int64_t *argmin, double *extra, int nthreads) {
    orc_tape t;
    tape_init(&t, nodes, n_nodes, consts, n_vars, roots, n_roots);
    if (nthreads < 1) nthreads = 1;
    int64_t count = k1 - k0;
    if (count < nthreads) nthreads = count > 0 ? (int)count : 1;
    orc_job *jobs = calloc((size_t)nthreads, sizeof(orc_job));
    double *reds = calloc((size_t)nthreads * 2 * n_roots, sizeof(double));
    pthread_t *th = calloc((size_t)nthreads, sizeof(pthread_t));
    for (int q = 0; q < nthreads; ++q) {
        orc_job *jb = &jobs[q];
        jb->t = &t; jb->box = box; jb->splits = splits; jb->ks = ks;
        jb->k0 = k0 + count * q / nthreads; jb->k1 = k0 + count * (q + 1) / nthreads;
        jb->kbase = k0;
        jb->mode = mode; jb->grad = grad; jb->count = count; jb->kinds = kinds;
        jb->per_sub = per_sub;                  /* [m][2][count], index q - k0 */
        jb->flags = flags;
        jb->red = reds + (size_t)q * 2 * n_roots;
    }
    if (nthreads == 1) bound_range(&jobs[0]);
    else {
        for (int q = 0; q < nthreads; ++q) pthread_create(&th[q], NULL, bound_range, &jobs[q]);
        for (int q = 0; q < nthreads; ++q) pthread_join(th[q], NULL);
    }
    int64_t am = -1;
    double best = INFINITY;
    for (int r = 0; r < n_roots; ++r) { reduced[2 * r] = INFINITY; reduced[2 * r + 1] = -INFINITY; }
    for (int q = 0; q < nthreads; ++q) {
        double *rd = jobs[q].red;
        if (jobs[q].k1 <= jobs[q].k0) continue;
        if (am < 0 || rd[0] < best) { best = rd[0]; am = jobs[q].argmin; }
        for (int r = 0; r < n_roots; ++r) {
            reduced[2 * r] = fmin(reduced[2 * r], rd[2 * r]);
            reduced[2 * r + 1] = fmax(reduced[2 * r + 1], rd[2 * r + 1]);
        }
    }
    if (argmin) *argmin = am;
    if (extra) {
        extra[0] = INFINITY;
        extra[1] = INFINITY;
        for (int q = 0; q < nthreads; ++q) {
            if (jobs[q].k1 <= jobs[q].k0) continue;
            extra[0] = fmin(extra[0], jobs[q].filtered_lo);
            extra[1] = fmin(extra[1], jobs[q].ub);
        }
    }
    free(jobs); free(reds); free(th);
    tape_free(&t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* exported: per-box evaluations for tests                                  */
/* ------------------------------------------------------------------------ */

/* NIE of every root on B boxes [B][n][2] -> out [B][m][2], flags [B] */
int orc_nie_boxes(const orc_node *nodes, int32_t n_nodes, const double *consts, int32_t n_vars,
                  const int32_t *roots, int32_t n_roots, int64_t B, const double *boxes,
                  double *out, uint32_t *flags) {
    orc_tape t;
    tape_init(&t, nodes, n_nodes, consts, n_vars, roots, n_roots);
    ivl *val = malloc(((size_t)n_nodes + 1) * sizeof(ivl));
    ivl X[256];
    for (int64_t b = 0; b < B; ++b) {
        for (int i = 0; i < n_vars; ++i) X[i] = I(boxes[(b * n_vars + i) * 2], boxes[(b * n_vars + i) * 2 + 1]);
        int bad = eval_values(&t, X, val);
        if (flags) flags[b] = bad ? 1u : 0u;
        for (int r = 0; r < n_roots; ++r) {
            out[(b * n_roots + r) * 2] = bad ? -INFINITY : val[roots[r]].lo;
            out[(b * n_roots + r) * 2 + 1] = bad ? INFINITY : val[roots[r]].hi;
        }
    }
    free(val);
    tape_free(&t);
    return 0;
}

/* interval gradient of root r on B boxes, forward (grad=0) or reverse (1) mode.
 * G [B][n][2]; flags [B]. */
int orc_gradient_boxes(const orc_node *nodes, int32_t n_nodes, const double *consts, int32_t n_vars,
                       const int32_t *roots, int32_t n_roots, int64_t B, const double *boxes, int32_t r,
                       int grad, double *G, uint32_t *flags) {
    orc_tape t;
    tape_init(&t, nodes, n_nodes, consts, n_vars, roots, n_roots);
    size_t N = (size_t)n_nodes + 1;
    ivl *val = malloc(N * sizeof(ivl)), *adj = malloc(N * sizeof(ivl));
    ivl *tan = malloc(N * ((size_t)n_vars + 1) * sizeof(ivl));
    ivl X[256], g[256];
    for (int64_t b = 0; b < B; ++b) {
        for (int i = 0; i < n_vars; ++i) X[i] = I(boxes[(b * n_vars + i) * 2], boxes[(b * n_vars + i) * 2 + 1]);
        int bad;
        if (grad == GRAD_FWD) {
            bad = eval_tangents(&t, X, val, tan);
            if (!bad) for (int j = 0; j < n_vars; ++j) g[j] = tan[(size_t)roots[r] * n_vars + j];
        } else {
            bad = eval_values(&t, X, val);
            if (!bad) gradient_rev(&t, r, val, adj, g);
        }
        if (flags) flags[b] = bad ? 1u : 0u;
        for (int j = 0; j < n_vars; ++j) {
            G[(b * n_vars + j) * 2] = bad ? -INFINITY : g[j].lo;
            G[(b * n_vars + j) * 2 + 1] = bad ? INFINITY : g[j].hi;
        }
    }
    free(val); free(adj); free(tan);
    tape_free(&t);
    return 0;
}

/* point evaluation: every root at degenerate boxes [x_b, x_b] -> f [B][m][2] */
int orc_eval_points(const orc_node *nodes, int32_t n_nodes, const double *consts, int32_t n_vars,
                    const int32_t *roots, int32_t n_roots, int64_t B, const double *x, double *f) {
    orc_tape t;
    tape_init(&t, nodes, n_nodes, consts, n_vars, roots, n_roots);
    ivl *val = malloc(((size_t)n_nodes + 1) * sizeof(ivl));
    ivl X[256];
    for (int64_t b = 0; b < B; ++b) {
        for (int i = 0; i < n_vars; ++i) X[i] = I(x[b * n_vars + i], x[b * n_vars + i]);
        int bad = eval_values(&t, X, val);
        for (int r = 0; r < n_roots; ++r) {
            f[(b * n_roots + r) * 2] = bad ? -INFINITY : val[roots[r]].lo;
            f[(b * n_roots + r) * 2 + 1] = bad ? INFINITY : val[roots[r]].hi;
        }
    }
    free(val);
    tape_free(&t);
    return 0;
}

/* vector-Jacobian product at points: one reverse sweep over all live nodes
 * seeded with adj[root_r] = [gout_r, gout_r]; gx [B][n][2] */
int orc_vjp_points(const orc_node *nodes, int32_t n_nodes, const double *consts, int32_t n_vars,
                   const int32_t *roots, int32_t n_roots, int64_t B, const double *x, const double *gout,
                   double *gx) {
    orc_tape t;
    tape_init(&t, nodes, n_nodes, consts, n_vars, roots, n_roots);
    size_t N = (size_t)n_nodes + 1;
    ivl *val = malloc(N * sizeof(ivl)), *adj = malloc(N * sizeof(ivl));
    ivl X[256], G[256];
    for (int64_t b = 0; b < B; ++b) {
        for (int i = 0; i < n_vars; ++i) X[i] = I(x[b * n_vars + i], x[b * n_vars + i]);
        int bad = eval_values(&t, X, val);
        for (int i = 0; i < n_nodes; ++i) adj[i] = I(0, 0);
        for (int j = 0; j < n_vars; ++j) G[j] = I(0, 0);
        for (int r = 0; r < n_roots; ++r) {
            double g = gout[b * n_roots + r];
            acc_to(&t, roots[r], I(g, g), adj, G);
        }
        if (!bad) reverse_sweep(&t, t.live, val, adj, G);
        for (int j = 0; j < n_vars; ++j) {
            gx[(b * n_vars + j) * 2] = bad ? -INFINITY : G[j].lo;
            gx[(b * n_vars + j) * 2 + 1] = bad ? INFINITY : G[j].hi;
        }
    }
    free(val); free(adj);
    tape_free(&t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* exported: adaptive partitioning (Sec. 3.1.2)                             */
/* ------------------------------------------------------------------------ */

/*
 * Largest uniform N with N^n <= budget, then +1 on one dimension at a time,
 * widest relative width w_i/s_i first (ties to the lower index), while the
 * count stays <= budget.  Writes splits[n]; returns the subdomain count.
 */
int64_t orc_adaptive_splits(int n, const double *widths, int64_t budget, int32_t *splits) {
    int64_t N = 1;
    for (;;) {
        int64_t p = 1;
        int over = 0;
        for (int i = 0; i < n; ++i) { p *= (N + 1); if (p > budget) { over = 1; break; } }
        if (over) break;
        ++N;
    }
    int64_t count = 1;
    for (int i = 0; i < n; ++i) { splits[i] = (int32_t)N; count *= N; }
    for (;;) {
        int best = -1;
        double bw = -1;
        for (int i = 0; i < n; ++i) {
            double rw = widths[i] / splits[i];
            if (rw > bw) { bw = rw; best = i; }
        }
        int64_t next = count / splits[best] * (splits[best] + 1);
        if (next > budget) break;
        count = next;
        splits[best] += 1;
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* constraint propagation (forward-backward bound tightening, FBBT)          */
/* ------------------------------------------------------------------------ */

/* The bound tightening the paper reports compatible with its method
 * (Sec. 3.2; its effect, Sec. 4.3): intervals of every live node on the box
 * (forward), the roots cut to their feasible ranges (g <= 0, h = 0, and the
 * objective <= ub), then in descending node order each operand intersected
 * with the outward-rounded inverse of its operation (backward); the box
 * shrinks to the intersection of its variables' nodes.  An empty
 * intersection proves the box infeasible.
 *
 * Forward, per op: the bounding extension of the op, except on a violated
 * domain (0 in a divisor, a negative sqrt argument, a non-positive log
 * argument), where the node is [-inf, +inf] (no information).
 * Backward, z = op(u, v), each result intersected with the current operand:
 *   add  U &= Z - V, then V &= Z - U        sub  U &= Z + V, then V &= U - Z
 *   mul  U &= Z / V if 0 not in V, then V &= Z / U if 0 not in U
 *   div  U &= Z * V, then V &= U / Z if 0 not in Z
 *   sqr  R = sqrt(Z & [0, inf)):  U &= R if lo(U) >= 0, -R if hi(U) <= 0,
 *        else [-hi(R), hi(R)]
 *   sqrt Z &= [0, inf), U &= sqr(Z)         exp  Z &= [0, inf), U &= log(Z)
 *        (the padded log; -inf below for lo(Z) = 0)
 *   log  U &= exp(Z)                         tanh Z &= [-1, 1], U &= atanh(Z)
 *        (libm in round-to-nearest widened by four ulps; +-inf at +-1)
 *   sin, cos  only the check that Z meets [-1, 1] (not monotone)
 * The inverse of an op is skipped where its own forward value carried no
 * information (a violated domain).  Rounds repeat forward and backward on
 * the tightened box. */

#define ORC_MAX_VARS 64

static ivl imeet(ivl a, ivl b) { return I(fmax(a.lo, b.lo), fmin(a.hi, b.hi)); }
static int iempty(ivl a) { return !(a.lo <= a.hi); }

static ivl iatanh(ivl z) {
    double lo = z.lo <= -1.0 ? -INFINITY : dn4(atanh(z.lo));
    double hi = z.hi >= 1.0 ? INFINITY : up4(atanh(z.hi));
    return I(lo, hi);
}

/* returns 1 when the box is proven infeasible; out receives the tightened box */
static int fbbt_box(const orc_tape *t, const int32_t *kinds, const double *box, double ub, int rounds,
                    double *out, ivl *val, uint8_t *info) {
    const int n = t->n_vars;
    ivl X[ORC_MAX_VARS];
    for (int j = 0; j < n; ++j) X[j] = I(box[2 * j], box[2 * j + 1]);
    for (int round = 0; round < rounds; ++round) {
        /* forward */
        for (int i = 0; i < t->n_nodes; ++i) {
            info[i] = 1;
            if (!t->live[i]) { val[i] = I(0, 0); continue; }
            const orc_node *nd = &t->nodes[i];
            ivl U = nd->op >= OP_ADD ? val[nd->a] : I(0, 0);
            ivl V = (nd->op >= OP_ADD && nd->op <= OP_DIV) ? val[nd->b] : I(0, 0);
            switch (nd->op) {
            case OP_VAR: val[i] = X[nd->a]; break;
            case OP_CONST: val[i] = I(t->consts[nd->a], t->consts[nd->a]); break;
            case OP_ADD: val[i] = iadd(U, V); break;
            case OP_SUB: val[i] = isub(U, V); break;
            case OP_MUL: val[i] = imul(U, V); break;
            case OP_DIV:
                if (V.lo <= 0 && V.hi >= 0) { info[i] = 0; val[i] = I(-INFINITY, INFINITY); }
                else val[i] = idiv(U, V);
                break;
            case OP_SQR: val[i] = isqr(U); break;
            case OP_SQRT:
                if (U.lo < 0) { info[i] = 0; val[i] = I(-INFINITY, INFINITY); }
                else val[i] = isqrt(U);
                break;
            case OP_EXP: val[i] = iexp(U); break;
            case OP_LOG:
                if (U.lo <= 0) { info[i] = 0; val[i] = I(-INFINITY, INFINITY); }
                else val[i] = ilog(U);
                break;
            case OP_TANH: val[i] = itanh(U); break;
            case OP_SIN: val[i] = isin(U); break;
            case OP_COS: val[i] = icos(U); break;
            }
        }
        /* the roots' feasible ranges */
        for (int r = 0; r < t->n_roots; ++r) {
            ivl *z = &val[t->roots[r]];
            if (kinds && kinds[r] == ORC_INEQ) *z = imeet(*z, I(-INFINITY, 0.0));
            else if (kinds && kinds[r] == ORC_EQ) *z = imeet(*z, I(0.0, 0.0));
            else if (r == 0 && ub < INFINITY) *z = imeet(*z, I(-INFINITY, ub));
        }
        /* backward */
        for (int i = t->n_nodes - 1; i >= 0; --i) {
            if (!t->live[i]) continue;
            if (iempty(val[i])) return 1;
            const orc_node *nd = &t->nodes[i];
            if (nd->op < OP_ADD || !info[i]) continue;
            ivl Z = val[i], *U = &val[nd->a], *V = nd->op <= OP_DIV ? &val[nd->b] : NULL, R;
            switch (nd->op) {
            case OP_ADD: *U = imeet(*U, isub(Z, *V)); *V = imeet(*V, isub(Z, *U)); break;
            case OP_SUB: *U = imeet(*U, iadd(Z, *V)); *V = imeet(*V, isub(*U, Z)); break;
            case OP_MUL:
                if (!(V->lo <= 0 && V->hi >= 0)) *U = imeet(*U, idiv(Z, *V));
                if (!iempty(*U) && !(U->lo <= 0 && U->hi >= 0)) *V = imeet(*V, idiv(Z, *U));
                break;
            case OP_DIV:
                *U = imeet(*U, imul(Z, *V));
                if (!(Z.lo <= 0 && Z.hi >= 0)) *V = imeet(*V, idiv(*U, Z));
                break;
            case OP_SQR:
                Z = imeet(Z, I(0.0, INFINITY));
                if (iempty(Z)) return 1;
                R = isqrt(Z);
                if (U->lo >= 0) *U = imeet(*U, R);
                else if (U->hi <= 0) *U = imeet(*U, I(-R.hi, -R.lo));
                else *U = imeet(*U, I(-R.hi, R.hi));
                break;
            case OP_SQRT:
                Z = imeet(Z, I(0.0, INFINITY));
                if (iempty(Z)) return 1;
                *U = imeet(*U, isqr(Z));
                break;
            case OP_EXP:
                Z = imeet(Z, I(0.0, INFINITY));
                if (iempty(Z)) return 1;
                if (Z.hi <= 0) return 1;                 /* exp > 0 */
                R = I(Z.lo <= 0 ? -INFINITY : dn2(log(Z.lo)), up2(log(Z.hi)));
                *U = imeet(*U, R);
                break;
            case OP_LOG: *U = imeet(*U, iexp(Z)); break;
            case OP_TANH:
                Z = imeet(Z, I(-1.0, 1.0));
                if (iempty(Z)) return 1;
                *U = imeet(*U, iatanh(Z));
                break;
            case OP_SIN: case OP_COS:
                if (iempty(imeet(Z, I(-1.0, 1.0)))) return 1;
                break;
            }
            if (iempty(*U) || (nd->op <= OP_DIV && iempty(*V))) return 1;
        }
        /* the box: every variable node of variable j narrows X_j */
        for (int i = 0; i < t->n_nodes; ++i)
            if (t->live[i] && t->nodes[i].op == OP_VAR) X[t->nodes[i].a] = imeet(X[t->nodes[i].a], val[i]);
        for (int j = 0; j < n; ++j)
            if (iempty(X[j])) return 1;
    }
    for (int j = 0; j < n; ++j) { out[2 * j] = X[j].lo; out[2 * j + 1] = X[j].hi; }
    return 0;
}

/* FBBT of N boxes; status[b] = 1 where a box is proven infeasible (out then undefined) */
int orc_fbbt(const orc_node *nodes, int32_t n_nodes, const double *consts, int32_t n_vars, const int32_t *roots,
             int32_t n_roots, const int32_t *kinds, int64_t N, const double *boxes, double ub, int32_t rounds,
             double *out, int32_t *status) {
    fesetround(FE_TONEAREST);
    orc_tape t;
    tape_init(&t, nodes, n_nodes, consts, n_vars, roots, n_roots);
    ivl *val = malloc(sizeof(ivl) * ((size_t)n_nodes + 1));
    uint8_t *info = malloc((size_t)n_nodes + 1);
    for (int64_t b = 0; b < N; ++b)
        status[b] = fbbt_box(&t, kinds, boxes + (size_t)b * n_vars * 2, ub, rounds, out + (size_t)b * n_vars * 2,
                             val, info);
    free(val);
    free(info);
    tape_free(&t);
    fesetround(FE_TONEAREST);
    return 0;
}
