/*
 * oracle.c -- plain FP64 CPU oracle for whole-population GP fitness evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it shares no code, header or table with the HIP library.
 *
 * What it computes (TensorGP, Sec. 3.1 "Genotype to Phenotype", Sec. 3.2
 * "Primitive Set" with Table 1, Sec. 4.1 for the RMSE objective):
 *   - every tree of the population is evaluated over every fitness case of an
 *     N-dimensional coordinate grid whose variables span [-1, 1] (Sec. 3.1);
 *   - each operator is applied with the protection rules of Table 1;
 *     trigonometric arguments are first multiplied by pi (Sec. 3.2);
 *   - the per-individual error against a target tensor is the root mean
 *     squared error (Sec. 4.1, Table 2) or the mean squared error.
 *
 * It walks each tree recursively, one fitness case at a time, in double
 * precision (mode O64).  For the parity contract it can also run, in the
 * same walk, (a) O32r: every operator computed in FP64 from its operands and
 * rounded to FP32, the way an FP32 tensor engine with correctly rounded
 * operators would compute, and (b) a first-order running error bound in the
 * manner of Wilkinson's forward error analysis: the bound of a node is the
 * sum over its operands of |partial derivative| x operand bound, plus the
 * rounding error an FP32 implementation of the operator may add (1 ulp for
 * add/sub/mult/div/sqrt/mdist/frac/mod, 4 ulp for the library functions).
 * At every operator with a discontinuity (protected division, log, sqrt,
 * pow, sign, step, if, mod, frac, tan, lerp) the walk also checks that the
 * O64 operand lies more than 4 bounds away from the discontinuity (or is
 * exactly on it with a zero bound) and that O32r falls on the same side.
 * A case is "stable" when those checks pass, O64 and O32r are finite, and
 * the bound of the root is at most 5e-6 * max(|O64|, 1), half the per-case
 * tolerance of the parity contract: to first order, no FP32 evaluation with
 * operators of the assumed accuracy can then miss O64 by more than that.
 *
 * Readings of points the paper leaves open (each one a deliberate choice):
 *   sin/cos are sin(pi x) and cos(pi x) (Table 1 prints them swapped);
 *   div(x, 0) = +0 for either sign of zero; log(x<0) = -1, log(0) = -inf;
 *   pow(0, 0) = 0, otherwise C99 pow; sqrt has arity 1 and sqrt(x<0) = 0;
 *   min/max are IEEE minNum/maxNum (a NaN operand yields the other one)
 *   with -0 ordered below +0 (so min(+0, -0) = -0 in either order);
 *   sign(NaN) = 0; clip(x, y, z) = max(min(x, z), y);
 *   mod is floored (result takes the divisor's sign), mod(x, 0) = 0;
 *   frac(x) = x - floor(x); if(x, y, z) = x != 0 ? y : z (NaN counts true);
 *   tan(x) = sin(pi x) / cos(pi x) with IEEE division;
 *   len(x, y) = the exact sqrt(x^2 + y^2) (hypot), NaN when an operand is
 *   NaN (the formula's value; C99 hypot would give +inf beside an infinite
 *   operand);
 *   warp(v, t0, t1) is a gather: v at the grid point whose axis-0 and axis-1
 *   positions t0, t1 name (nearest point, halves rounded up, clamped, NaN
 *   giving the first point; a third axis keeps its own point);
 *   or/xor/and act on 32-bit integers made from the operands by truncation
 *   toward zero with saturation (NaN gives 0), as Table 1's footnote asks
 *   for a conversion to integers;
 *   coordinate k along an axis of n points is the FP32 rounding of
 *   lo + (hi - lo) * k / (n - 1) computed in FP64 (lo when n == 1),
 *   axes row-major with the last axis fastest; axis 0 is x, 1 is y, 2 is z.
 * Any non-finite squared error makes an individual's fitness +inf.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint8_t op, var;
    uint16_t pad;
    float value;
} orc_token;

/* Opcodes in the order of the paper's Table 1 (terminals first). */
enum {
    OV_VAR, OV_CONST,
    OV_ADD, OV_SUB, OV_MULT, OV_DIV,
    OV_SIN, OV_COS, OV_TAN,
    OV_EXP, OV_LOG, OV_POW,
    OV_MIN, OV_MAX, OV_MDIST, OV_NEG,
    OV_SQRT, OV_SIGN, OV_ABS, OV_CLIP,
    OV_MOD, OV_FRAC, OV_IF,
    OV_STEP, OV_SSTEP, OV_SSTEPP, OV_LEN, OV_LERP,
    OV_OR, OV_XOR, OV_AND,
    OV_WARP,
    OV_COUNT
};

static const int orc_arity[OV_COUNT] = {
    0, 0,
    2, 2, 2, 2,
    1, 1, 1,
    1, 1, 2,
    2, 2, 2, 1,
    1, 1, 1, 3,
    2, 1, 3,
    1, 1, 1, 2, 3,
    2, 2, 2,
    3,
};

#define ORC_MAX_DIM 3

typedef struct {
    uint8_t op, var;
    float value;
    int32_t kid[3];
} onode;

typedef struct {
    onode *n;
    int32_t count; /* root is n[count-1] */
} otree;

/* ---------------------------------------------------------------- parsing */

/* Returns 0 on success, -1 on a malformed tree (bad opcode, var, arity). */
static int build_tree(const orc_token *t, int64_t len, int ndim, otree *out)
{
    out->n = NULL;
    out->count = 0;
    if (len <= 0)
        return -1;
    onode *n = (onode *)malloc(sizeof(onode) * (size_t)len);
    int32_t *stk = (int32_t *)malloc(sizeof(int32_t) * (size_t)len);
    if (!n || !stk) {
        free(n);
        free(stk);
        return -1;
    }
    int64_t sp = 0;
    for (int64_t i = 0; i < len; i++) {
        int op = t[i].op;
        if (op >= OV_COUNT)
            goto bad;
        if (op == OV_VAR && t[i].var >= ndim)
            goto bad;
        int a = orc_arity[op];
        if (sp < a)
            goto bad;
        n[i].op = (uint8_t)op;
        n[i].var = t[i].var;
        n[i].value = t[i].value;
        n[i].kid[0] = n[i].kid[1] = n[i].kid[2] = -1;
        for (int j = a - 1; j >= 0; j--)
            n[i].kid[j] = stk[--sp];
        stk[sp++] = (int32_t)i;
    }
    if (sp != 1)
        goto bad;
    free(stk);
    out->n = n;
    out->count = (int32_t)len;
    return 0;
bad:
    free(n);
    free(stk);
    return -1;
}

/* ------------------------------------------------------ operator semantics */

/* sin(pi x) and cos(pi x) without rounding pi: x is reduced exactly to
 * t = x - n/2 with |t| <= 1/4 and n = rint(2x), then the quadrant n mod 4
 * picks +-sin(pi t) or +-cos(pi t).  Exact at every multiple of 1/2. */
static void sincospi64(double x, double *s, double *c)
{
    if (!isfinite(x)) {
        *s = *c = NAN;
        return;
    }
    if (fabs(x) >= 9007199254740992.0) { /* 2^53: every double is an even integer */
        *s = 0.0;
        *c = 1.0;
        return;
    }
    double n = rint(2.0 * x);
    double t = x - 0.5 * n; /* exact */
    double st = sin(M_PI * t), ct = cos(M_PI * t);
    long q = (long)fmod(n, 4.0);
    if (q < 0)
        q += 4;
    switch (q) {
    case 0: *s = st;  *c = ct;  break;
    case 1: *s = ct;  *c = -st; break;
    case 2: *s = -st; *c = -ct; break;
    default: *s = -ct; *c = st; break;
    }
    /* zeros of sin(pi x) and cos(pi x) are returned as +0 */
    if (*s == 0.0) *s = 0.0;
    if (*c == 0.0) *c = 0.0;
}

/* IEEE minNum / maxNum (a NaN operand yields the other one) with -0 ordered
 * below +0, so the result does not depend on the operand order. */
static double min_num(double a, double b)
{
    if (a == 0.0 && b == 0.0)
        return signbit(a) ? a : b;
    return fmin(a, b);
}

static double max_num(double a, double b)
{
    if (a == 0.0 && b == 0.0)
        return signbit(a) ? b : a;
    return fmax(a, b);
}

static double floor_mod(double x, double y)
{
    if (y == 0.0)
        return 0.0;
    double r = fmod(x, y);
    if (r != 0.0 && ((r < 0.0) != (y < 0.0)))
        r += y;
    return r;
}

/* The integer a bitwise operator works on: NaN gives 0, other values are
 * truncated toward zero and saturated to the 32-bit range. */
static int32_t to_i32(double x)
{
    if (isnan(x))
        return 0;
    if (x >= 2147483648.0)
        return INT32_MAX;
    if (x <= -2147483649.0)
        return INT32_MIN;
    return (int32_t)trunc(x);
}

static int is_integral(double v)
{
    return isfinite(v) && floor(v) == v;
}

/* Applies operator op to a, b, c (unused operands ignored) in FP64.
 * *br receives the side of the operator's discontinuity the operands fall on
 * (0 for operators without one); NaN-free integers or floors, compared by
 * value across evaluation variants. */
static double apply(int op, double a, double b, double c, double *br)
{
    double s, co;
    *br = 0.0;
    switch (op) {
    case OV_ADD: return a + b;
    case OV_SUB: return a - b;
    case OV_MULT:
        /* an infinite factor times a finite one: the sign (or NaN at 0) of
         * the finite one decides the result */
        if (isinf(a) != isinf(b))
            *br = (double)(((isinf(a) ? b : a) > 0.0) - ((isinf(a) ? b : a) < 0.0));
        return a * b;
    case OV_DIV:
        *br = (b == 0.0);
        return b == 0.0 ? 0.0 : a / b;
    case OV_SIN: sincospi64(a, &s, &co); return s;
    case OV_COS: sincospi64(a, &s, &co); return co;
    case OV_TAN:
        *br = isfinite(a) ? floor(a + 0.5) : -1.0;
        sincospi64(a, &s, &co);
        return s / co;
    case OV_EXP: return exp(a);
    case OV_LOG:
        *br = isnan(a) ? 3 : (a < 0.0 ? 0 : (a == 0.0 ? 1 : 2));
        return a < 0.0 ? -1.0 : log(a);
    case OV_POW:
        if (isnan(a) || isnan(b)) *br = 5;
        else if (a == 0.0 && b == 0.0) *br = 0;
        else if (a == 0.0) *br = (b > 0.0 ? 1 : 6) + (signbit(a) ? 10 : 0);  /* 0^b: +-0 or +-inf */
        else if (isinf(b)) *br = fabs(a) < 1.0 ? 7 : (fabs(a) == 1.0 ? 8 : 9);
        else if (a < 0.0) *br = is_integral(b) ? 2 : 3;
        else *br = 4;
        return (a == 0.0 && b == 0.0) ? 0.0 : pow(a, b);
    case OV_MIN: return min_num(a, b);
    case OV_MAX: return max_num(a, b);
    case OV_MDIST: return (a + b) / 2.0;
    case OV_NEG: return -a;
    case OV_SQRT:
        *br = (a < 0.0);
        return a < 0.0 ? 0.0 : sqrt(a);
    case OV_SIGN:
        *br = isnan(a) ? 3 : (a < 0.0 ? 0 : (a == 0.0 ? 1 : 2));
        return (double)((a > 0.0) - (a < 0.0));
    case OV_ABS: return fabs(a);
    case OV_CLIP: return max_num(min_num(a, c), b);
    case OV_MOD:
        if (b == 0.0 || isnan(a) || isnan(b)) *br = 1e308;
        else if (isinf(b)) *br = (a != 0.0 && ((a < 0.0) != (b < 0.0))) ? -1.0 : 0.0;  /* a or +-inf */
        else *br = floor(a / b);
        return floor_mod(a, b);
    case OV_FRAC:
        *br = isfinite(a) ? floor(a) : -1.0;
        return a - floor(a);
    case OV_IF:
        *br = (a != 0.0);
        return a != 0.0 ? b : c;
    case OV_STEP:
        *br = (a < 0.0);
        return a < 0.0 ? -1.0 : 1.0;
    case OV_SSTEP: return a * a * (3.0 - 2.0 * a);
    case OV_SSTEPP: return a * a * a * (a * (6.0 * a - 15.0) + 10.0);
    case OV_LEN: return isnan(a) || isnan(b) ? NAN : hypot(a, b);
    case OV_LERP:
        *br = isfinite(c) ? floor(c) : -1.0;
        return a + (b - a) * (c - floor(c));
    case OV_OR:
    case OV_XOR:
    case OV_AND: {
        const int32_t ia = to_i32(a), ib = to_i32(b);
        *br = (double)ia * 4294967296.0 + (double)(uint32_t)ib;
        return (double)(op == OV_OR ? (ia | ib) : (op == OV_XOR ? (ia ^ ib) : (ia & ib)));
    }
    }
    return NAN;
}

/* ------------------------------------------------------------ the domain */

typedef struct {
    int ndim;
    int64_t shape[ORC_MAX_DIM];
    int64_t stride[ORC_MAX_DIM];
    double lo[ORC_MAX_DIM], hi[ORC_MAX_DIM];
    float *coord[ORC_MAX_DIM];
} odomain;

static int make_domain(int ndim, const int64_t *shape, const double *lo, const double *hi, odomain *d)
{
    memset(d, 0, sizeof(*d));
    if (ndim < 1 || ndim > ORC_MAX_DIM)
        return -1;
    d->ndim = ndim;
    int64_t st = 1;
    for (int k = ndim - 1; k >= 0; k--) {
        if (shape[k] < 1)
            return -1;
        d->shape[k] = shape[k];
        d->stride[k] = st;
        st *= shape[k];
    }
    for (int k = 0; k < ndim; k++) {
        d->lo[k] = lo[k];
        d->hi[k] = hi[k];
        d->coord[k] = (float *)malloc(sizeof(float) * (size_t)shape[k]);
        for (int64_t i = 0; i < shape[k]; i++) {
            double v = shape[k] == 1 ? lo[k] : lo[k] + (hi[k] - lo[k]) * (double)i / (double)(shape[k] - 1);
            d->coord[k][i] = (float)v;
        }
    }
    return 0;
}

static void free_domain(odomain *d)
{
    for (int k = 0; k < ORC_MAX_DIM; k++)
        free(d->coord[k]);
}

static void case_coords(const odomain *d, int64_t c, double *xyz)
{
    for (int k = 0; k < d->ndim; k++) {
        int64_t i = (c / d->stride[k]) % d->shape[k];
        xyz[k] = (double)d->coord[k][i];
    }
}

/* ---------------------------------------------------------------- warp */

/* warp(v, t0, t1) (Sec. 3.2, Table 1) read as a gather: the value at a case is
 * v at the grid point that t0 and t1 name along axes 0 and 1, each the
 * nearest point of its axis (position u = (t - lo)(n - 1)/(hi - lo) rounded
 * half up, clamped to the axis, NaN giving point 0); a third axis keeps the
 * case's own point, and a 1-D domain ignores t1.  Index of axis k: */
static int64_t warp_axis(const odomain *d, int k, double t)
{
    const int64_t n = d->shape[k];
    if (n == 1)
        return 0;
    const double u = (t - d->lo[k]) * ((double)(n - 1) / (d->hi[k] - d->lo[k])) + 0.5;
    const double w = fmin(fmax(u, 0.0), (double)(n - 1)); /* fmax(NaN, 0) = 0 */
    return (int64_t)floor(w);
}

/* Coordinates of the point warp reads, from the current case's coordinates. */
static void warp_coords(const odomain *d, double t0, double t1, const double *xyz, double *out)
{
    out[0] = d->coord[0][warp_axis(d, 0, t0)];
    if (d->ndim > 1)
        out[1] = d->coord[1][warp_axis(d, 1, t1)];
    if (d->ndim > 2)
        out[2] = xyz[2];
}

/* Is the rounding of axis k's position clear of its steps by MARGIN bounds,
 * given the bound e of t?  The steps are at the integers 1 .. n - 1 of
 * u = position + 1/2; the FP32 evaluation of u adds up to 3 ulp of u. */
static int warp_axis_clear(const odomain *d, int k, double t, double e);

/* ------------------------------------------------------- the tree walkers */

static double ev64(const odomain *d, const onode *n, int32_t i, const double *xyz)
{
    const onode *p = &n[i];
    if (p->op == OV_VAR)
        return xyz[p->var];
    if (p->op == OV_CONST)
        return (double)p->value;
    double a = 0.0, b = 0.0, c = 0.0, br;
    int ar = orc_arity[p->op];
    if (p->op == OV_WARP) {
        double at[3];
        warp_coords(d, ev64(d, n, p->kid[1], xyz), ev64(d, n, p->kid[2], xyz), xyz, at);
        return ev64(d, n, p->kid[0], at);
    }
    a = ev64(d, n, p->kid[0], xyz);
    if (ar > 1)
        b = ev64(d, n, p->kid[1], xyz);
    if (ar > 2)
        c = ev64(d, n, p->kid[2], xyz);
    return apply(p->op, a, b, c, &br);
}

static int same_branch(double a, double b)
{
    return a == b || (isnan(a) && isnan(b));
}

/* Rounding error an FP32 implementation of the operator may add, relative. */
#define U_CR 1.1920928955078125e-07   /* 2^-23: one ulp, correctly rounded ops */
#define U_LIB 4.76837158203125e-07    /* 2^-21: four ulp, library functions */
#define MARGIN 4.0
/* A first-order bound is trusted while the change it allows stays within
 * this fraction of the scale on which the operator bends (a period, a
 * unit of an exponent, the factors' own size); beyond it the case is not
 * checked. */
#define LINEAR 0.0625
/* FLT_MAX plus half an ulp: FP32 rounding sends magnitudes from here on to inf */
#define FLT_OVERFLOW 3.4028235677973366e+38

/* Rounding an FP32 implementation of an operator may add to a result of
 * magnitude av, for a relative accuracy u: below the normal range FP32
 * values are spaced 2^-149 apart whatever their size, so the error is u
 * times 2^-126 there (an exact zero stays exact, as in the relative model). */
static double rnd(double u, double av)
{
    return u == 0.0 || av == 0.0 ? 0.0 : u * (av > 0x1p-126 ? av : 0x1p-126);
}

static double contrib(double deriv, double e)
{
    return e == 0.0 ? 0.0 : fabs(deriv) * e;
}

/* Is x at least MARGIN bounds away from the point p (or exactly on it with a
 * zero bound)? */
static int clear_of(double x, double p, double e)
{
    if (e == 0.0)
        return 1;
    return fabs(x - p) > MARGIN * e;
}

/* Bound of min or max (result val) of x and y with bounds ex, ey: when
 * the operands are further apart than their bounds allow to close, every
 * FP32 evaluation picks the same one and the result carries its bound;
 * otherwise either may be picked (the operators are continuous, so the
 * larger bound covers both). */
static double select_bound(double x, double ex, double y, double ey, double val)
{
    if (fabs(x - y) > ex + ey)
        return val == x ? ex : ey;
    return ex > ey ? ex : ey;
}

static double dist_to_int(double x)
{
    return fabs(x - rint(x));
}

/* One node in O64 (v), O32r (r) and the running bound (e); *ok is cleared
 * when a discontinuity is too close or O32r falls on another side. */
static int warp_axis_clear(const odomain *d, int k, double t, double e)
{
    const int64_t n = d->shape[k];
    if (n == 1 || !isfinite(t))
        return 1;
    const double scale = (double)(n - 1) / (d->hi[k] - d->lo[k]);
    const double u = (t - d->lo[k]) * scale + 0.5;
    const double eu = fabs(scale) * e + 3.0 * U_CR * (fabs(u) + 1.0);
    if (u < -MARGIN * eu || u > (double)(n - 1) + MARGIN * eu)
        return 1; /* clamped */
    return dist_to_int(u) > MARGIN * eu;
}

static void evb(const odomain *d, const onode *n, int32_t i, const double *xyz, double *v, double *r,
                double *e, int *ok)
{
    const onode *p = &n[i];
    if (p->op == OV_VAR) {
        *v = *r = xyz[p->var];
        *e = 0.0;
        return;
    }
    if (p->op == OV_CONST) {
        *v = *r = (double)p->value;
        *e = 0.0;
        return;
    }
    double kv[3] = {0, 0, 0}, kr[3] = {0, 0, 0}, ke[3] = {0, 0, 0};
    int ar = orc_arity[p->op];
    if (p->op == OV_WARP) {
        /* the coordinates first; then v at the point they name (O64's point;
         * O32r must name the same one) */
        for (int j = 1; j < 3; j++)
            evb(d, n, p->kid[j], xyz, &kv[j], &kr[j], &ke[j], ok);
        for (int k = 0; k < d->ndim && k < 2; k++) {
            if (warp_axis(d, k, kv[1 + k]) != warp_axis(d, k, kr[1 + k]) ||
                !warp_axis_clear(d, k, kv[1 + k], ke[1 + k]))
                *ok = 0;
        }
        double at[3];
        warp_coords(d, kv[1], kv[2], xyz, at);
        evb(d, n, p->kid[0], at, v, r, e, ok);
        return;
    }
    for (int j = 0; j < ar; j++) {
        evb(d, n, p->kid[j], xyz, &kv[j], &kr[j], &ke[j], ok);
        /* an operand finite in FP64 but beyond FP32's range is +-inf in any
         * FP32 evaluation, so O64 above it describes none of them */
        if (isfinite(kv[j]) && fabs(kv[j]) >= FLT_OVERFLOW)
            *ok = 0;
    }
    double br0, br1;
    const double a = kv[0], b = kv[1], c = kv[2];
    const double ea = ke[0], eb = ke[1], ec = ke[2];
    const double val = apply(p->op, a, b, c, &br0);
    *r = (double)(float)apply(p->op, kr[0], kr[1], kr[2], &br1);
    if (!same_branch(br0, br1))
        *ok = 0;
    *v = val;
    double err = 0.0;
    const double av = fabs(val);
    /* A correctly rounded operator whose operands are exact (zero bound)
     * adds no error when its exact result is an FP32 value: rounding a
     * representable value returns it.  (The FP64 result of FP32 operands is
     * then that exact value: FP64 rounding cannot land on an FP32 value a
     * non-representable quotient or root misses by more than 2^-48.) */
    const int exact_in = ea == 0.0 && eb == 0.0 && ec == 0.0;
    const double ucr = exact_in && (double)(float)val == val ? 0.0 : U_CR;
    double s, co;
    switch (p->op) {
    case OV_ADD:
    case OV_SUB: err = ea + eb + rnd(ucr, av); break;
    case OV_MULT:
        if ((isinf(a) && !clear_of(b, 0.0, eb)) || (isinf(b) && !clear_of(a, 0.0, ea))) *ok = 0;
        err = contrib(b, ea) + contrib(a, eb) + rnd(ucr, av);
        if (ea * eb > LINEAR * err) *ok = 0;   /* the product of the two errors is not negligible */
        break;
    case OV_DIV:
        if (b == 0.0) {
            if (eb != 0.0) *ok = 0;
            err = 0.0;
        } else {
            if (!clear_of(b, 0.0, eb)) *ok = 0;
            err = contrib(1.0 / b, ea) + contrib(a / (b * b), eb) + rnd(ucr, av);
        }
        break;
    /* sin(pi a) and cos(pi a) of an exact multiple of 1/2 are exactly 0 or
     * +-1 (the argument reduction is exact, see sincospi64) */
    case OV_SIN:
        sincospi64(a, &s, &co);
        if (M_PI * ea > LINEAR) *ok = 0;       /* phase error not small against the period */
        err = contrib(M_PI * co, ea) + rnd(exact_in && rint(2.0 * a) == 2.0 * a ? 0.0 : U_LIB, av);
        break;
    case OV_COS:
        sincospi64(a, &s, &co);
        if (M_PI * ea > LINEAR) *ok = 0;
        err = contrib(M_PI * s, ea) + rnd(exact_in && rint(2.0 * a) == 2.0 * a ? 0.0 : U_LIB, av);
        break;
    case OV_TAN:
        sincospi64(a, &s, &co);
        if (!clear_of(fabs(a - floor(a)), 0.5, ea)) *ok = 0;
        if (M_PI * ea > LINEAR) *ok = 0;
        err = contrib(M_PI / (co * co), ea) + rnd(U_LIB, av);
        break;
    case OV_EXP:
        if (ea > LINEAR) *ok = 0;              /* relative change e^ea - 1 not first-order */
        err = contrib(val, ea) + rnd(U_LIB, av);
        break;
    case OV_LOG:
        if (!clear_of(a, 0.0, ea)) *ok = 0;
        err = a > 0.0 ? contrib(1.0 / a, ea) + rnd(U_LIB, av) : 0.0;
        break;
    case OV_POW:
        if (a == 0.0 && b == 0.0) {
            if (ea != 0.0 || eb != 0.0) *ok = 0;
            err = 0.0;
            break;
        }
        if (!clear_of(a, 0.0, ea)) *ok = 0;
        if (a == 0.0 && !clear_of(b, 0.0, eb)) *ok = 0;          /* 0^b: 0 or +inf by the sign of b */
        if (isinf(b) && !clear_of(fabs(a), 1.0, ea)) *ok = 0;    /* a^(+-inf) jumps at |a| = 1 */
        if (a < 0.0 && eb != 0.0 && dist_to_int(b) <= MARGIN * eb) *ok = 0;
        if (a != 0.0 && isfinite(val)) {
            /* the exponent b log|a| must move by little for a first-order bound */
            if (contrib(b / a, ea) + (a > 0.0 ? contrib(log(a), eb) : 0.0) > LINEAR) *ok = 0;
            err = contrib(b * val / a, ea) + (a > 0.0 ? contrib(val * log(a), eb) : 0.0) + rnd(U_LIB, av);
        }
        break;
    case OV_MIN:
    case OV_MAX: err = select_bound(a, ea, b, eb, val); break;
    case OV_MDIST: err = 0.5 * (ea + eb) + rnd(ucr, av); break;
    case OV_NEG:
    case OV_ABS: err = ea; break;
    case OV_SQRT:
        if (!clear_of(a, 0.0, ea)) *ok = 0;
        err = a > 0.0 ? contrib(0.5 / sqrt(a), ea) + rnd(ucr, av) : 0.0;
        break;
    case OV_SIGN:
    case OV_STEP:
        if (!clear_of(a, 0.0, ea)) *ok = 0;
        err = 0.0;
        break;
    case OV_CLIP: {
        const double m = min_num(a, c);
        err = select_bound(m, select_bound(a, ea, c, ec, m), b, eb, val);
        break;
    }
    case OV_MOD:
        if (b == 0.0) {
            if (eb != 0.0) *ok = 0;
            err = 0.0;
        } else if (isinf(b)) {
            if (isfinite(a) && !clear_of(a, 0.0, ea)) *ok = 0;  /* a, or +-inf past 0 */
            err = ea;
        } else {
            const double q = a / b;
            const double eq = (ea + fabs(q) * eb) / fabs(b);
            if (eq != 0.0 && dist_to_int(q) <= MARGIN * eq) *ok = 0;
            err = ea + contrib(floor(q), eb) + rnd(ucr, av);
        }
        break;
    case OV_FRAC:
        if (ea != 0.0 && dist_to_int(a) <= MARGIN * ea) *ok = 0;
        err = ea + rnd(ucr, av);
        break;
    case OV_IF:
        if (!clear_of(a, 0.0, ea)) *ok = 0;
        err = a != 0.0 ? eb : ec;
        break;
    case OV_SSTEP:
        if (ea > LINEAR * LINEAR / (1.0 + fabs(a))) *ok = 0;   /* curvature 6 - 12a */
        err = contrib(6.0 * a - 6.0 * a * a, ea) + rnd(U_LIB, av);
        break;
    case OV_SSTEPP:
        if (ea > LINEAR * LINEAR / (1.0 + a * a * a * a)) *ok = 0;
        err = contrib(30.0 * a * a * (a - 1.0) * (a - 1.0), ea) + rnd(U_LIB, av);
        break;
    case OV_LEN:
        err = val == 0.0 ? ea + eb : contrib(a / val, ea) + contrib(b / val, eb) + rnd(U_LIB, av);
        break;
    case OV_LERP: {
        const double fz = c - floor(c);
        if (ec != 0.0 && dist_to_int(c) <= MARGIN * ec) *ok = 0;
        err = contrib(1.0 - fz, ea) + contrib(fz, eb) + contrib(b - a, ec) + rnd(U_LIB, av);
        break;
    }
    case OV_OR:
    case OV_XOR:
    case OV_AND:
        /* truncation jumps at every non-zero integer */
        if (ea != 0.0 && fabs(rint(a)) >= 1.0 && dist_to_int(a) <= MARGIN * ea) *ok = 0;
        if (eb != 0.0 && fabs(rint(b)) >= 1.0 && dist_to_int(b) <= MARGIN * eb) *ok = 0;
        /* the integer result is the same (checked above); only its
         * rounding to FP32 can add error */
        err = (double)(float)val == val ? 0.0 : rnd(U_CR, av);
        break;
    }
    if (!isfinite(val))
        err = 0.0;   /* an exact special value; its class is checked instead */
    else if (!isfinite(err))
        *ok = 0;
    else if (!clear_of(av, FLT_OVERFLOW, err))
        *ok = 0;     /* FP32 rounds to +-inf from FLT_OVERFLOW on: finite or not is undecided */
    *e = err;
}

static int nonfinite_class(double v)
{
    if (isnan(v)) return 1;
    if (isinf(v)) return v > 0 ? 2 : 3;
    return 0;
}

/*
 * Evaluate trees over fitness cases.
 *   tokens/offsets: n_roots postfix trees (tree r = tokens[offsets[r]..offsets[r+1]) ).
 *   ndim/shape/lo/hi: the coordinate grid.
 *   cases: n_cases case indices (row-major, last axis fastest), or NULL for
 *          all cases in order (then n_cases must equal the grid size).
 *   v64:   out [n_roots][n_cases] O64 values (required).
 *   v32r:  out [n_roots][n_cases] O32r values, or NULL.
 *   stab:  out [n_roots][n_cases] flags, or NULL: bit0 = stable finite case,
 *          bit1 = O32r and the FP32 rounding of O64 are non-finite of one
 *          class, clear of every discontinuity (that class is then required),
 *          bit2 = a finite case clear of every discontinuity (O64 and O32r
 *          finite, O32r on O64's side of each) whose bound exceeds the
 *          stable limit but not 1/16 of max(|O64|, 1), with O32r within the
 *          bound (plus the stable limit) of O64: any FP32 evaluation
 *          with operators of the assumed accuracy is then within the bound
 *          of O64 to first order, and the bound is small enough that the
 *          neglected second-order terms stay a few percent of it.
 *   ebound: out [n_roots][n_cases] running error bound of the root, or NULL.
 *   When any of v32r, stab, ebound is given the checked walk runs; otherwise
 *   only O64.
 * Returns 0, or -(1 + r) when tree r is malformed, or -1000000000 on bad args.
 */
int orc_eval(const orc_token *tokens, const int64_t *offsets, int64_t n_roots,
             int ndim, const int64_t *shape, const double *lo, const double *hi,
             const int64_t *cases, int64_t n_cases,
             double *v64, double *v32r, uint8_t *stab, double *ebound, int nthreads)
{
    odomain d;
    if (make_domain(ndim, shape, lo, hi, &d) != 0)
        return -1000000000;
    int64_t total = 1;
    for (int k = 0; k < ndim; k++)
        total *= shape[k];
    if (!cases && n_cases != total) {
        free_domain(&d);
        return -1000000000;
    }
    otree *trees = (otree *)calloc((size_t)(n_roots > 0 ? n_roots : 1), sizeof(otree));
    int rc = 0;
    for (int64_t r = 0; r < n_roots; r++) {
        if (build_tree(tokens + offsets[r], offsets[r + 1] - offsets[r], ndim, &trees[r]) != 0) {
            rc = (int)(-(1 + r));
            break;
        }
    }
    if (rc == 0) {
        int four = (v32r != NULL) || (stab != NULL) || (ebound != NULL);
        int64_t work = n_roots * n_cases;
#ifdef _OPENMP
        if (nthreads > 0)
            omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
        for (int64_t w = 0; w < work; w += 256) {
            int64_t end = w + 256 < work ? w + 256 : work;
            for (int64_t q = w; q < end; q++) {
                int64_t r = q / n_cases, ci = q % n_cases;
                int64_t c = cases ? cases[ci] : ci;
                double xyz[ORC_MAX_DIM] = {0, 0, 0};
                case_coords(&d, c, xyz);
                const otree *t = &trees[r];
                if (!four) {
                    v64[q] = ev64(&d, t->n, t->count - 1, xyz);
                    continue;
                }
                double v, r32, e;
                int ok = 1;
                evb(&d, t->n, t->count - 1, xyz, &v, &r32, &e, &ok);
                v64[q] = v;
                if (v32r)
                    v32r[q] = r32;
                if (ebound)
                    ebound[q] = e;
                if (stab) {
                    uint8_t f = 0;
                    const double sc = fabs(v) > 1.0 ? fabs(v) : 1.0;
                    if (ok && isfinite(v) && isfinite(r32) && e <= 5e-6 * sc && fabs(r32 - v) <= 5e-6 * sc)
                        f |= 1;
                    const int cl = nonfinite_class(r32);
                    const int cv = nonfinite_class((double)(float)v);
                    if (ok && isfinite(v) && isfinite(r32) && !(f & 1) && e <= 0.0625 * sc &&
                        fabs(r32 - v) <= e + 5e-6 * sc)
                        f |= 4;
                    if (ok && cl && cl == cv &&
                        (!isfinite(v) || fabs(v) - e > 3.4028235677973366e38 * (1.0 + 5.9604644775390625e-08)))
                        f |= 2;
                    stab[q] = f;
                }
            }
        }
    }
    (void)nthreads;
    for (int64_t r = 0; r < n_roots; r++)
        free(trees[r].n);
    free(trees);
    free_domain(&d);
    return rc;
}

/* Coordinate table of one axis, for tests of the grid convention. */
int orc_coords(int64_t n, double lo, double hi, float *out)
{
    if (n < 1)
        return -1;
    for (int64_t i = 0; i < n; i++)
        out[i] = (float)(n == 1 ? lo : lo + (hi - lo) * (double)i / (double)(n - 1));
    return 0;
}

/*
 * Fitness per individual from per-case values (Sec. 4.1: RMSE against the
 * target).  values: [n_ind * n_ch][n_cases] FP64, tree-major (individual i,
 * channel ch is row i * n_ch + ch).  target: [n_ch][n_cases] FP32.
 * Sums (v - t)^2 in FP64 in index order over channels then cases; loss 0
 * gives sqrt(sum / N), loss 1 gives sum / N, with N = n_ch * n_cases.
 * Any non-finite term makes the fitness +inf.
 */
int orc_fitness(const double *values, const float *target, int64_t n_ind, int n_ch,
                int64_t n_cases, int loss, double *out)
{
    if (n_ch < 1 || n_cases < 1 || (loss != 0 && loss != 1))
        return -1;
    double N = (double)n_ch * (double)n_cases;
    for (int64_t i = 0; i < n_ind; i++) {
        double s = 0.0;
        int bad = 0;
        for (int ch = 0; ch < n_ch; ch++) {
            const double *v = values + (i * n_ch + ch) * n_cases;
            const float *t = target + (int64_t)ch * n_cases;
            for (int64_t c = 0; c < n_cases; c++) {
                double e = v[c] - (double)t[c];
                double q = e * e;
                if (!isfinite(q))
                    bad = 1;
                s += q;
            }
        }
        out[i] = bad ? INFINITY : (loss == 0 ? sqrt(s / N) : s / N);
    }
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
