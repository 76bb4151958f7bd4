/*
 * CPU oracle for Pauli propagation -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU library.
 *
 * Two plain, slow, FP64 routines:
 *
 *  1. orc_sv_*: dense state-vector simulation, the textbook definition of
 *     <O> = <0|U^dag O U|0> (Sec. I: a PQC U(theta) of m gates acting on
 *     |0...0>; Sec. II-A: measurement read from the final state).
 *
 *  2. orc_propagate: scalar propagation of a weighted Pauli sum (Sec. II-A,
 *     the stabilizer written as sum_j lambda_j P_j with real lambda), one gate
 *     at a time, following the paper's gate rules:
 *       - single-qubit gates H, S, R_x, R_y, R_z act on the weight vector
 *         w = [w_I, w_X, w_Y, w_Z] of the acted-on qubit exactly as Table I
 *         prints them (the paper's forward map  P -> g P g^dag);
 *       - CX maps the (control, target) letter pair by the 16-entry list of
 *         Sec. III-C (control = first letter), including XZ <-> -YY;
 *       - after every gate the set is expanded and reduced: equal strings are
 *         merged by summing their weights (Sec. III-B, Examples 3 and 4,
 *         eq. (7)), with no pruning -- zero weights are kept.
 *     direction 0 (Heisenberg, observable propagation): gates g_m ... g_1,
 *       each applied through its inverse g^dag P g, built from Table I as
 *       H^-1 = H, S^-1 = S S S, R(theta)^-1 = R(-theta), CX^-1 = CX.
 *     direction 1 (Schroedinger, generator evolution of eq. (1)): gates
 *       g_1 ... g_m applied with Table I directly.
 *     The number of term updates U = sum over gates of the set size entering
 *     that gate is returned alongside.
 *
 * Conventions: bit q of x/z is qubit q; I=(0,0) X=(1,0) Y=(1,1) Z=(0,1);
 * Y is the Hermitian Pauli; R_sigma(theta) = exp(-i theta sigma/2).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OP_H = 0, OP_S = 1, OP_CX = 2, OP_RX = 3, OP_RY = 4, OP_RZ = 5 };
enum { L_I = 0, L_X = 1, L_Y = 2, L_Z = 3 }; /* the paper's letter order */

/* ------------------------------------------------------------------------ */
/* 1. dense state vector                                                    */
/* ------------------------------------------------------------------------ */

static void sv_apply_1q(int n, double complex *psi, int q, const double complex u[2][2]) {
    const uint64_t dim = 1ull << n, bit = 1ull << q;
    for (uint64_t b = 0; b < dim; ++b) {
        if (b & bit) continue;
        double complex a0 = psi[b], a1 = psi[b | bit];
        psi[b] = u[0][0] * a0 + u[0][1] * a1;
        psi[b | bit] = u[1][0] * a0 + u[1][1] * a1;
    }
}

static void sv_apply_cx(int n, double complex *psi, int c, int t) {
    const uint64_t dim = 1ull << n, bc = 1ull << c, bt = 1ull << t;
    for (uint64_t b = 0; b < dim; ++b) {
        if ((b & bc) && !(b & bt)) {
            double complex tmp = psi[b];
            psi[b] = psi[b | bt];
            psi[b | bt] = tmp;
        }
    }
}

/* Gate matrices: H, S = diag(1, i), R_sigma(theta) = exp(-i theta sigma / 2). */
static void gate_matrix(int op, double th, double complex u[2][2]) {
    const double r = 1.0 / sqrt(2.0), c = cos(th / 2.0), s = sin(th / 2.0);
    switch (op) {
    case OP_H: u[0][0] = r; u[0][1] = r; u[1][0] = r; u[1][1] = -r; break;
    case OP_S: u[0][0] = 1; u[0][1] = 0; u[1][0] = 0; u[1][1] = I; break;
    case OP_RX: u[0][0] = c; u[0][1] = -I * s; u[1][0] = -I * s; u[1][1] = c; break;
    case OP_RY: u[0][0] = c; u[0][1] = -s; u[1][0] = s; u[1][1] = c; break;
    default: /* OP_RZ */
        u[0][0] = cexp(-I * th / 2.0); u[0][1] = 0; u[1][0] = 0; u[1][1] = cexp(I * th / 2.0);
        break;
    }
}

/* Runs g_1 ... g_m on |0...0>; psi (2^n complex, as re/im pairs) is output. */
int orc_sv_run(int n, int64_t m, const uint8_t *op, const int32_t *q0, const int32_t *q1,
               const int32_t *param, const double *theta, double *psi_out) {
    if (n < 1 || n > 26) return -1;
    const uint64_t dim = 1ull << n;
    double complex *psi = calloc(dim, sizeof(double complex));
    if (!psi) return -2;
    psi[0] = 1.0;
    for (int64_t g = 0; g < m; ++g) {
        if (op[g] == OP_CX) {
            sv_apply_cx(n, psi, q0[g], q1[g]);
        } else {
            double complex u[2][2];
            double th = (op[g] >= OP_RX) ? theta[param[g]] : 0.0;
            gate_matrix(op[g], th, u);
            sv_apply_1q(n, psi, q0[g], u);
        }
    }
    for (uint64_t b = 0; b < dim; ++b) {
        psi_out[2 * b] = creal(psi[b]);
        psi_out[2 * b + 1] = cimag(psi[b]);
    }
    free(psi);
    return 0;
}

/* <psi| sum_k c_k P_k |psi>.  P(x,z)|b> = i^{|x&z|} (-1)^{|b&z|} |b xor x>. */
double orc_sv_expval(int n, const double *psi_in, int64_t nt, const uint64_t *x,
                     const uint64_t *z, const double *coef) {
    const uint64_t dim = 1ull << n;
    const double complex *psi = (const double complex *)psi_in;
    double total = 0.0;
    for (int64_t k = 0; k < nt; ++k) {
        double complex acc = 0.0;
        int ny = __builtin_popcountll(x[k] & z[k]) & 3;
        double complex ph = (ny == 0) ? 1.0 : (ny == 1) ? I : (ny == 2) ? -1.0 : -I;
        for (uint64_t b = 0; b < dim; ++b) {
            double sgn = (__builtin_popcountll(b & z[k]) & 1) ? -1.0 : 1.0;
            acc += conj(psi[b ^ x[k]]) * ph * sgn * psi[b];
        }
        total += coef[k] * creal(acc);
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* 2. scalar Pauli propagation                                              */
/* ------------------------------------------------------------------------ */

typedef struct { uint64_t x, z; double c; } term_t;
typedef struct { term_t *v; int64_t n, cap; } tset_t;

static int ts_push(tset_t *s, uint64_t x, uint64_t z, double c) {
    if (s->n == s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 64;
        term_t *nv = realloc(s->v, (size_t)nc * sizeof(term_t));
        if (!nv) return -1;
        s->v = nv;
        s->cap = nc;
    }
    s->v[s->n].x = x; s->v[s->n].z = z; s->v[s->n].c = c;
    s->n++;
    return 0;
}

/* canonical order: by z, then by x */
static int term_cmp(const void *a, const void *b) {
    const term_t *p = a, *q = b;
    if (p->z != q->z) return p->z < q->z ? -1 : 1;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    return 0;
}

/* reduce(): sort, then sum the weights of equal strings; zeros are kept.
 * qsort is not stable, so equal strings are summed in an unspecified order;
 * for reproducible rounding the run is sorted on (key, arrival) instead. */
typedef struct { term_t t; int64_t arrival; } tagged_t;
static int tagged_cmp(const void *a, const void *b) {
    const tagged_t *p = a, *q = b;
    int r = term_cmp(&p->t, &q->t);
    if (r) return r;
    return p->arrival < q->arrival ? -1 : (p->arrival > q->arrival);
}

static int ts_reduce(tset_t *s) {
    if (s->n == 0) return 0;
    tagged_t *tmp = malloc((size_t)s->n * sizeof(tagged_t));
    if (!tmp) return -1;
    for (int64_t i = 0; i < s->n; ++i) { tmp[i].t = s->v[i]; tmp[i].arrival = i; }
    qsort(tmp, (size_t)s->n, sizeof(tagged_t), tagged_cmp);
    int64_t w = 0;
    for (int64_t i = 0; i < s->n; ++i) {
        if (w > 0 && s->v[w - 1].x == tmp[i].t.x && s->v[w - 1].z == tmp[i].t.z)
            s->v[w - 1].c += tmp[i].t.c;
        else
            s->v[w++] = tmp[i].t;
    }
    s->n = w;
    free(tmp);
    return 0;
}

static int letter_of(uint64_t x, uint64_t z, int q) {
    int xb = (int)((x >> q) & 1), zb = (int)((z >> q) & 1);
    if (!xb && !zb) return L_I;
    if (xb && !zb) return L_X;
    if (xb && zb) return L_Y;
    return L_Z;
}

static void set_letter(uint64_t *x, uint64_t *z, int q, int L) {
    uint64_t m = 1ull << q;
    *x &= ~m;
    *z &= ~m;
    if (L == L_X || L == L_Y) *x |= m;
    if (L == L_Z || L == L_Y) *z |= m;
}

/* Table I: the output weight vector w' = A w of each single-qubit gate.
 *   H : [w0,  w3, -w2,  w1]
 *   S : [w0, -w2,  w1,  w3]
 *   Rx: [w0,  w1,  w2 c - w3 s,  w2 s + w3 c]
 *   Ry: [w0,  w1 c + w3 s,  w2,  w3 c - w1 s]
 *   Rz: [w0,  w1 c - w2 s,  w2 c + w1 s,  w3]
 * A[out][in]; live[out][in] marks entries that are not identically zero as a
 * function of theta, so a cos/sin entry is kept even where it evaluates to 0. */
static void table1(int op, double th, double A[4][4], int live[4][4]) {
    const double c = cos(th), s = sin(th);
    memset(A, 0, 16 * sizeof(double));
    memset(live, 0, 16 * sizeof(int));
    A[0][0] = 1; live[0][0] = 1;
    switch (op) {
    case OP_H:
        A[1][3] = 1; A[2][2] = -1; A[3][1] = 1;
        live[1][3] = live[2][2] = live[3][1] = 1;
        break;
    case OP_S:
        A[1][2] = -1; A[2][1] = 1; A[3][3] = 1;
        live[1][2] = live[2][1] = live[3][3] = 1;
        break;
    case OP_RX:
        A[1][1] = 1;
        A[2][2] = c; A[2][3] = -s;
        A[3][2] = s; A[3][3] = c;
        live[1][1] = live[2][2] = live[2][3] = live[3][2] = live[3][3] = 1;
        break;
    case OP_RY:
        A[1][1] = c; A[1][3] = s;
        A[2][2] = 1;
        A[3][1] = -s; A[3][3] = c;
        live[1][1] = live[1][3] = live[2][2] = live[3][1] = live[3][3] = 1;
        break;
    default: /* OP_RZ */
        A[1][1] = c; A[1][2] = -s;
        A[2][1] = s; A[2][2] = c;
        A[3][3] = 1;
        live[1][1] = live[1][2] = live[2][1] = live[2][2] = live[3][3] = 1;
        break;
    }
}

/* one forward application of a single-qubit gate to every term, then reduce */
static int apply_1q_forward(tset_t *s, int op, int q, double th) {
    double A[4][4];
    int live[4][4];
    table1(op, th, A, live);
    tset_t out = {0};
    for (int64_t i = 0; i < s->n; ++i) {
        term_t t = s->v[i];
        int L = letter_of(t.x, t.z, q);
        for (int Lo = 0; Lo < 4; ++Lo) {
            if (!live[Lo][L]) continue;
            uint64_t x = t.x, z = t.z;
            set_letter(&x, &z, q, Lo);
            if (ts_push(&out, x, z, t.c * A[Lo][L])) { free(out.v); return -1; }
        }
    }
    free(s->v);
    *s = out;
    return ts_reduce(s);
}

/* Sec. III-C: CX on (control, target) letters.  Pairs swap; XZ <-> -YY. */
static const char *CX_LIST[][2] = {
    {"XI", "XX"}, {"IY", "ZY"}, {"YI", "YX"}, {"IZ", "ZZ"}, {"XY", "YZ"},
    {"II", "II"}, {"IX", "IX"}, {"ZI", "ZI"}, {"ZX", "ZX"}, {"XZ", "-YY"},
};

static int letter_from_char(char ch) {
    return ch == 'X' ? L_X : ch == 'Y' ? L_Y : ch == 'Z' ? L_Z : L_I;
}

static void cx_table(int out_c[4][4], int out_t[4][4], double sign[4][4]) {
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) { out_c[a][b] = -1; out_t[a][b] = -1; sign[a][b] = 0; }
    for (size_t k = 0; k < sizeof(CX_LIST) / sizeof(CX_LIST[0]); ++k) {
        const char *l = CX_LIST[k][0], *r = CX_LIST[k][1];
        double sg = 1.0;
        if (r[0] == '-') { sg = -1.0; ++r; }
        int lc = letter_from_char(l[0]), lt = letter_from_char(l[1]);
        int rc = letter_from_char(r[0]), rt = letter_from_char(r[1]);
        out_c[lc][lt] = rc; out_t[lc][lt] = rt; sign[lc][lt] = sg;
        out_c[rc][rt] = lc; out_t[rc][rt] = lt; sign[rc][rt] = sg;
    }
}

static int apply_cx(tset_t *s, int c, int t) {
    int oc[4][4], ot[4][4];
    double sg[4][4];
    cx_table(oc, ot, sg);
    for (int64_t i = 0; i < s->n; ++i) {
        term_t *p = &s->v[i];
        int lc = letter_of(p->x, p->z, c), lt = letter_of(p->x, p->z, t);
        set_letter(&p->x, &p->z, c, oc[lc][lt]);
        set_letter(&p->x, &p->z, t, ot[lc][lt]);
        p->c *= sg[lc][lt];
    }
    return ts_reduce(s);
}

static int apply_gate(tset_t *s, int op, int q0, int q1, double th, int heisenberg) {
    if (op == OP_CX) return apply_cx(s, q0, q1);
    if (!heisenberg) return apply_1q_forward(s, op, q0, th);
    /* g^dag P g is the forward map of g^-1 */
    if (op == OP_H) return apply_1q_forward(s, OP_H, q0, 0.0);
    if (op == OP_S) {
        for (int k = 0; k < 3; ++k)
            if (apply_1q_forward(s, OP_S, q0, 0.0)) return -1;
        return 0;
    }
    return apply_1q_forward(s, op, q0, -th);
}

/*
 * Propagates the observable (nt_in terms) through the circuit.
 *   direction 0: Heisenberg (g_m first, inverse maps); 1: Schroedinger.
 * Outputs: the final set in canonical order (at most cap_out terms are
 * written; *n_out is the full size), *updates = sum_g |set entering g|, and
 * the return value is sum of c over strings with x = 0 (i.e. <0|O'|0>).
 * A negative *n_out reports an allocation failure.
 */
double orc_propagate(int n, int64_t m, const uint8_t *op, const int32_t *q0, const int32_t *q1,
                     const int32_t *param, const double *theta, int direction, int64_t nt_in,
                     const uint64_t *x, const uint64_t *z, const double *coef, int64_t cap_out,
                     uint64_t *x_out, uint64_t *z_out, double *c_out, int64_t *n_out,
                     int64_t *updates) {
    (void)n;
    tset_t s = {0};
    int64_t U = 0;
    for (int64_t k = 0; k < nt_in; ++k)
        if (ts_push(&s, x[k], z[k], coef[k])) goto fail;
    if (ts_reduce(&s)) goto fail;
    for (int64_t k = 0; k < m; ++k) {
        int64_t g = direction == 0 ? m - 1 - k : k;
        double th = (op[g] >= OP_RX) ? theta[param[g]] : 0.0;
        U += s.n;
        if (apply_gate(&s, op[g], q0[g], q1[g], th, direction == 0)) goto fail;
    }
    double ev = 0.0;
    for (int64_t i = 0; i < s.n; ++i)
        if (s.v[i].x == 0) ev += s.v[i].c;
    for (int64_t i = 0; i < s.n && i < cap_out; ++i) {
        x_out[i] = s.v[i].x; z_out[i] = s.v[i].z; c_out[i] = s.v[i].c;
    }
    *n_out = s.n;
    *updates = U;
    free(s.v);
    return ev;
fail:
    free(s.v);
    *n_out = -1;
    *updates = U;
    return NAN;
}
