/*
 * fmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the
 * hierarchical 2D fast multipole method for the complex logarithm kernel
 *     Phi_j = sum_i u_i log(y_j - x_i)          (paper Sec. 2, eqs. 1-2)
 * on the three tilings of Luo & Duraiswami, "Alternative tilings for the fast
 * multipole method on the plane" (arXiv:1204.3105): the square quadtree, the
 * hexagonal septree (base-7 GBT addresses, Sec. 5) and the triangle-quadtree
 * (Sec. 6).  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code, header, table or helper
 * with the GPU library; the only thing both sides see is the seeded input.
 *
 * The paper omits the expansion and translation operators (end of Sec. 2).
 * They are taken from Greengard & Rokhlin, "A fast algorithm for particle
 * simulations", J. Comput. Phys. 73 (1987), Lemmas 2.1-2.5 (multipole
 * expansion, multipole shift, multipole-to-local, local shift, evaluation).
 *
 * Readings of passages that are silent, ambiguous or garbled (all listed in
 * the design notes of the repository):
 *  - NeighborsE4 (Sec. 4) prints an intersection with Neighbors(n, l); the
 *    interaction list is the set DIFFERENCE (children of the parent
 *    neighbourhood minus the cell and its own neighbours), which is the only
 *    reading that yields the P4 counts 27 / 42 / 39 of the cost table.
 *  - Complex log branch: Log z = ln|z| + i atan2(Im z, Re z) with a -0
 *    imaginary part taken as +0, so the negative real axis maps to +pi.
 *    Every difference is formed target minus source.
 *  - A source and a target with bitwise-equal coordinates do not interact.
 *  - Strengths u_i are real.
 *  - Septree: digit k in 1..6 is the lattice direction at angle
 *    k*60deg - 30deg (the CellCenter polar formula at j = 0); digit 1 is the
 *    b axis and digit 2 the c axis of the change of basis in Sec. 5.
 *  - Triangle-quadtree: the lattice angle in CellIndex uses the parent's
 *    orientation; "t = n_7" in CellIndex is read as n_4.
 *  - Centres are formed from exact integer lattice coordinates (quadtree:
 *    cell indices; septree: zero-extension relation of Sec. 5 in integers;
 *    triangle-quadtree: the F(t,i) translations, whose cosines and sines are
 *    0, +-1/2, +-sqrt(3)/2, +-1, accumulated in integer units).
 *  - Ties in nearest-centre decisions: strict "<" over the candidates in the
 *    order the paper lists them.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum { TIL_QUAD = 0, TIL_SEPT = 1, TIL_TRI = 2 };

/* Geometry of one tree.
 *   quadtree : (ox, oy) lower-left corner of the root square, size = side.
 *   septree  : (ox, oy) centre of leaf hexagon 0, size = leaf hexagon
 *              circumradius r (adjacent leaf centres are r*sqrt(3) apart).
 *   triangle : (ox, oy) centroid of the upright root triangle, size = leaf
 *              triangle circumradius r (root inradius = 2^(L-1) r).       */
typedef struct {
    int32_t tiling;
    int32_t L;
    double ox, oy;
    double size;
} orc_geom;

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int64_t ipow(int64_t b, int e)
{
    int64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

static int tiling_base(int tiling) { return tiling == TIL_SEPT ? 7 : 4; }

/* Canonical principal logarithm: arg in (-pi, pi], -0 imaginary part -> +0. */
static cplx log_canon(cplx z)
{
    double re = creal(z), im = cimag(z);
    if (im == 0.0) im = 0.0;
    return CMPLX(log(hypot(re, im)), atan2(im, re));
}

/* ===================================================================== */
/* Quadtree (Sec. 4): Morton Z order, child digit = 2*ybit + xbit.        */
/* ===================================================================== */

static int64_t quad_interleave(int64_t ix, int64_t iy, int l)
{
    int64_t key = 0;
    for (int b = 0; b < l; ++b) {
        key |= ((ix >> b) & 1) << (2 * b);
        key |= ((iy >> b) & 1) << (2 * b + 1);
    }
    return key;
}

static void quad_split(int64_t key, int l, int64_t *ix, int64_t *iy)
{
    int64_t x = 0, y = 0;
    for (int b = 0; b < l; ++b) {
        x |= ((key >> (2 * b)) & 1) << b;
        y |= ((key >> (2 * b + 1)) & 1) << b;
    }
    *ix = x;
    *iy = y;
}

static int64_t quad_cell_index(const orc_geom *g, double x, double y, int l)
{
    double h = ldexp(g->size, -l);
    double fx = floor((x - g->ox) / h);
    double fy = floor((y - g->oy) / h);
    double n = ldexp(1.0, l);
    if (!(fx >= 0.0 && fx < n && fy >= 0.0 && fy < n)) return -1;
    return quad_interleave((int64_t)fx, (int64_t)fy, l);
}

static void quad_center(const orc_geom *g, int64_t key, int l, double *cx, double *cy)
{
    int64_t ix, iy;
    quad_split(key, l, &ix, &iy);
    double h = ldexp(g->size, -l);
    *cx = g->ox + ((double)ix + 0.5) * h;
    *cy = g->oy + ((double)iy + 0.5) * h;
}

/* Cells sharing a vertex: the eight integer offsets that stay inside. */
static int quad_neighbors(int64_t key, int l, int64_t *out)
{
    int64_t ix, iy, n = (int64_t)1 << l;
    quad_split(key, l, &ix, &iy);
    int cnt = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            int64_t jx = ix + dx, jy = iy + dy;
            if (jx < 0 || jy < 0 || jx >= n || jy >= n) continue;
            out[cnt++] = quad_interleave(jx, jy, l);
        }
    return cnt;
}

/* ===================================================================== */
/* Septree (Sec. 5): base-7 Generalized Balanced Ternary.                 */
/* ===================================================================== */

/* Unit-addition table of Sec. 5.1 exactly as printed: entry [a][b] is the
 * GBT sum a (+) b written as a base-7 numeral (tens digit = carry).        */
static const int gbt_table[7][7] = {
    {0, 1, 2, 3, 4, 5, 6},
    {1, 63, 15, 2, 0, 6, 64},
    {2, 15, 14, 26, 3, 0, 1},
    {3, 2, 26, 25, 31, 4, 0},
    {4, 0, 3, 31, 36, 42, 5},
    {5, 6, 0, 4, 42, 41, 53},
    {6, 64, 1, 0, 5, 53, 52},
};

#define GBT_MAXD 40
typedef struct { int d[GBT_MAXD]; } gbt_num; /* d[0] = least significant */

static void gbt_from_key(int64_t key, gbt_num *n)
{
    memset(n, 0, sizeof(*n));
    for (int i = 0; i < GBT_MAXD && key > 0; ++i) {
        n->d[i] = (int)(key % 7);
        key /= 7;
    }
}

/* Value of the digits, or -1 if a digit at position >= maxd is nonzero. */
static int64_t gbt_to_key(const gbt_num *n, int maxd)
{
    for (int i = maxd; i < GBT_MAXD; ++i)
        if (n->d[i]) return -1;
    int64_t key = 0;
    for (int i = maxd - 1; i >= 0; --i) key = key * 7 + n->d[i];
    return key;
}

/* Add the unit digit d at position pos, propagating carries by the table. */
static int gbt_add_unit(gbt_num *n, int pos, int d)
{
    while (d != 0) {
        if (pos >= GBT_MAXD) return -1;
        int v = gbt_table[n->d[pos]][d];
        n->d[pos] = v % 10;
        d = v / 10;
        ++pos;
    }
    return 0;
}

/* a <- a (+) b, digit by digit. */
static int gbt_add(gbt_num *a, const gbt_num *b)
{
    for (int i = 0; i < GBT_MAXD; ++i)
        if (b->d[i] && gbt_add_unit(a, i, b->d[i])) return -1;
    return 0;
}

/* GBT index of m copies of the unit digit dpos (digit dneg when m < 0),
 * by double-and-add with (+). */
static int gbt_multiple(int64_t m, int dpos, int dneg, gbt_num *out)
{
    memset(out, 0, sizeof(*out));
    int d = dpos;
    if (m < 0) {
        m = -m;
        d = dneg;
    }
    gbt_num pw;
    memset(&pw, 0, sizeof(pw));
    pw.d[0] = d;
    while (m) {
        if ((m & 1) && gbt_add(out, &pw)) return -1;
        m >>= 1;
        if (m) {
            gbt_num t = pw;
            if (gbt_add(&pw, &t)) return -1;
        }
    }
    return 0;
}

/* Integer lattice coordinates (b, c) of the unit digits (angle k*60-30 deg). */
static const int sept_unit_b[7] = {0, 1, 0, -1, -1, 0, 1};
static const int sept_unit_c[7] = {0, 0, 1, 1, 0, -1, -1};

/* Lattice vector of digit d followed by k zeros, by the zero-extension
 * relation  d0^k = d0^(k-1) (+) e0^(k-1) (+) e0^(k-1),  e = 1 + (d mod 6). */
static void sept_zero_ext(int d, int k, int64_t *b, int64_t *c)
{
    int64_t vb[7], vc[7], nb[7], nc[7];
    for (int e = 0; e < 7; ++e) {
        vb[e] = sept_unit_b[e];
        vc[e] = sept_unit_c[e];
    }
    for (int s = 0; s < k; ++s) {
        for (int e = 1; e < 7; ++e) {
            int f = 1 + (e % 6);
            nb[e] = vb[e] + 2 * vb[f];
            nc[e] = vc[e] + 2 * vc[f];
        }
        for (int e = 1; e < 7; ++e) {
            vb[e] = nb[e];
            vc[e] = nc[e];
        }
    }
    *b = vb[d];
    *c = vc[d];
}

/* Lattice coordinates of cell key at level l (leaf units). */
static void sept_lattice(const orc_geom *g, int64_t key, int l, int64_t *B, int64_t *C)
{
    int64_t sb = 0, sc = 0;
    for (int pos = 0; pos < l; ++pos) {
        int d = (int)(key % 7);
        key /= 7;
        if (d) {
            int64_t b, c;
            sept_zero_ext(d, pos + (g->L - l), &b, &c);
            sb += b;
            sc += c;
        }
    }
    *B = sb;
    *C = sc;
}

static void sept_center(const orc_geom *g, int64_t key, int l, double *cx, double *cy)
{
    const double r = g->size, s3 = sqrt(3.0);
    int64_t B, C;
    sept_lattice(g, key, l, &B, &C);
    *cx = g->ox + (3.0 * r * (double)B) / 2.0;
    *cy = g->oy + (r * s3 * (2.0 * (double)C + (double)B)) / 2.0;
}

/* CellCenter in the polar form of eq. (septreecenter); test use only. */
static void sept_center_polar(const orc_geom *g, int64_t key, int l, double *cx, double *cy)
{
    const double r = g->size;
    int digits[GBT_MAXD], nd = 0;
    int64_t k = key;
    while (k > 0) {
        digits[nd++] = (int)(k % 7);
        k /= 7;
    }
    /* t_1 is the left-most significant digit; |t| = nd. */
    double x = 0.0, y = 0.0;
    for (int i = 1; i <= nd; ++i) {
        int ti = digits[nd - i];
        if (!ti) continue;
        int j = (nd - i) + (g->L - l);
        double th = j * atan(sqrt(3.0) / 2.0) + ti * M_PI / 3.0 - M_PI / 6.0;
        double R = r * sqrt(3.0) * pow(sqrt(7.0), j);
        x += R * cos(th);
        y += R * sin(th);
    }
    *cx = g->ox + x;
    *cy = g->oy + y;
}

/* Leaf key of the lattice point b * (digit-1 unit) + c * (digit-2 unit):
 * the two GBT multiples summed with (+); -1 if it needs more than L digits,
 * i.e. lies outside the root aggregate. */
static int64_t sept_key_of_lattice(const orc_geom *g, int64_t b, int64_t c)
{
    gbt_num u, v;
    if (gbt_multiple(b, 1, 4, &u)) return -1;
    if (gbt_multiple(c, 2, 5, &v)) return -1;
    if (gbt_add(&u, &v)) return -1;
    return gbt_to_key(&u, g->L);
}

/* CellIndex at the leaf level (Sec. 5): change of basis, four candidate
 * lattice points, nearest by squared distance, then its GBT index. */
static int64_t sept_leaf_index(const orc_geom *g, double x, double y)
{
    const double r = g->size, s3 = sqrt(3.0);
    double X = x - g->ox, Y = y - g->oy;
    double b = (2.0 * X) / (3.0 * r);
    double c = (s3 * Y - X) / (3.0 * r);
    if (!isfinite(b) || !isfinite(c)) return -1;
    double cb[4] = {floor(b), ceil(b), floor(b), ceil(b)};
    double cc[4] = {floor(c), floor(c), ceil(c), ceil(c)};
    int best = 0;
    double bestd = INFINITY;
    for (int i = 0; i < 4; ++i) {
        double px = (3.0 * r * cb[i]) / 2.0;
        double py = (r * s3 * (2.0 * cc[i] + cb[i])) / 2.0;
        double dx = X - px, dy = Y - py;
        double d2 = dx * dx + dy * dy;
        if (d2 < bestd) {
            bestd = d2;
            best = i;
        }
    }
    if (fabs(cb[best]) > 1e12 || fabs(cc[best]) > 1e12) return -1;
    return sept_key_of_lattice(g, (int64_t)cb[best], (int64_t)cc[best]);
}

/* Neighbours of a level-l cell (Sec. 5): the cells whose centres sit one
 * level-l lattice step away, i.e. the centre plus the lattice vector of each
 * unit digit followed by L - l zeros.  Each such point is a level-l centre,
 * so its leaf index ends in L - l zero digits; points outside the root
 * aggregate have no index and are dropped. */
static int sept_neighbors(const orc_geom *g, int64_t key, int l, int64_t *out)
{
    int64_t B, C;
    sept_lattice(g, key, l, &B, &C);
    const int64_t scale = ipow(7, g->L - l);
    int cnt = 0;
    for (int d = 1; d <= 6; ++d) {
        int64_t db, dc;
        sept_zero_ext(d, g->L - l, &db, &dc);
        int64_t k = sept_key_of_lattice(g, B + db, C + dc);
        if (k < 0) continue;
        if (k % scale) abort(); /* a level-l lattice point always ends in zeros */
        out[cnt++] = k / scale;
    }
    return cnt;
}

/* ===================================================================== */
/* Triangle-quadtree (Sec. 6).  Types 0 centre, 1 vertical, 2 left,      */
/* 3 right.  Centres in integer units: x = U * (sqrt(3)/2) r,            */
/* y = V * r/2 (leaf circumradius r).                                    */
/* ===================================================================== */

static int tq_digit(int64_t key, int l, int i) /* t_i, i = 1 is left-most */
{
    return (int)((key >> (2 * (l - i))) & 3);
}

/* isUp(t, l) = 2[(parity(t) + l - |t| + 1) mod 2] - 1, t = n_4 written
 * without leading zeros, parity = number of zero digits mod 2. */
static int tq_is_up(int64_t key, int l)
{
    int nd = 0, zeros = 0;
    int64_t k = key;
    do {
        if ((k & 3) == 0) ++zeros;
        ++nd;
        k >>= 2;
    } while (k > 0);
    int par = zeros & 1;
    int m = (par + l - nd + 1) % 2;
    if (m < 0) m += 2;
    return 2 * m - 1;
}

/* Integer-unit centre (U, V) of a cell, by the F(t, i) translations. */
static void tq_center_units(const orc_geom *g, int64_t key, int l, int64_t *U, int64_t *V)
{
    int64_t u = 0, v = 0;
    for (int i = 1; i <= l; ++i) {
        int ti = tq_digit(key, l, i);
        if (!ti) continue;
        int o = tq_is_up(key >> (2 * (l - i)), i);
        int64_t R = (int64_t)1 << (g->L - i);
        if (ti == 1) {
            v += 2 * o * R;
        } else if (ti == 2) {
            u -= R;
            v -= o * R;
        } else {
            u += R;
            v -= o * R;
        }
    }
    *U = u;
    *V = v;
}

static void tq_center(const orc_geom *g, int64_t key, int l, double *cx, double *cy)
{
    const double r = g->size, s3 = sqrt(3.0);
    int64_t U, V;
    tq_center_units(g, key, l, &U, &V);
    double ax = (s3 * r) / 2.0, ay = r / 2.0;
    *cx = g->ox + (double)U * ax;
    *cy = g->oy + (double)V * ay;
}

/* CellIndex (Sec. 6): top-down, nearest of the four child centres. */
static int64_t tq_cell_index(const orc_geom *g, double x, double y, int l)
{
    const double r = g->size, s3 = sqrt(3.0);
    double X = x - g->ox, Y = y - g->oy;
    double rho0 = ldexp(r, g->L - 1);
    double hs3 = s3 / 2.0;
    if (!isfinite(X) || !isfinite(Y)) return -1;
    if (Y < -rho0 || hs3 * X + 0.5 * Y > rho0 || -hs3 * X + 0.5 * Y > rho0) return -1;
    double ax = (s3 * r) / 2.0, ay = r / 2.0;
    int64_t U = 0, V = 0, key = 0;
    int up = 1;
    for (int i = 1; i <= l; ++i) {
        int64_t R = (int64_t)1 << (g->L - i);
        int64_t cu[4] = {U, U, U - R, U + R};
        int64_t cv[4] = {V, V + 2 * up * R, V - up * R, V - up * R};
        int best = 0;
        double bestd = INFINITY;
        for (int t = 0; t < 4; ++t) {
            double px = (double)cu[t] * ax, py = (double)cv[t] * ay;
            double dx = X - px, dy = Y - py;
            double d2 = dx * dx + dy * dy;
            if (d2 < bestd) {
                bestd = d2;
                best = t;
            }
        }
        U = cu[best];
        V = cv[best];
        if (best == 0) up = -up;
        key = key * 4 + best;
    }
    return key;
}

/* Cell at level l whose centroid is the integer-unit point (U, V), by
 * CellIndex of that point; 0 if it lies outside the root triangle.  A
 * lattice centroid is an inradius away from every edge, far beyond
 * rounding, so CellIndex returns the triangle it is the centroid of. */
static int tq_cell_at(const orc_geom *g, int64_t U, int64_t V, int l, int64_t *out)
{
    const double r = g->size, s3 = sqrt(3.0);
    double ax = (s3 * r) / 2.0, ay = r / 2.0;
    int64_t k = tq_cell_index(g, g->ox + (double)U * ax, g->oy + (double)V * ay, l);
    if (k < 0) return 0;
    int64_t U2, V2;
    tq_center_units(g, k, l, &U2, &V2);
    if (U2 != U || V2 != V) abort(); /* not a lattice centroid of level l */
    *out = k;
    return 1;
}

/* The cell across one edge (Sec. 6; direction 0 = left, 1 = right, 2 =
 * vertical).  A triangle of orientation o (+1 up) and circumradius s units
 * has its vertices at (0, 2os), (-s, -os), (s, -os) from its centroid; the
 * triangle across the edge opposite a vertex is its mirror image in that
 * edge, with the centroid at minus that vertex offset: vertical (0, -2os),
 * left (-s, os), right (s, os). */
static int tq_adjacent(const orc_geom *g, int64_t key, int l, int dir, int64_t *out)
{
    int64_t U, V;
    tq_center_units(g, key, l, &U, &V);
    const int64_t s = (int64_t)1 << (g->L - l);
    const int o = tq_is_up(key, l);
    const int64_t dU[3] = {-s, s, 0}, dV[3] = {o * s, o * s, -2 * o * s};
    return tq_cell_at(g, U + dU[dir], V + dV[dir], l, out);
}

/* Neighbours (Sec. 6): every cell sharing a vertex with the cell.  Six
 * triangles meet at each lattice vertex, their centroids one circumradius
 * from it in the directions -90 + 60k degrees: (0, -2s), (s, -s), (s, s),
 * (0, 2s), (-s, s), (-s, -s) in integer units.  Over the three vertices,
 * less the cell itself and repeats, that is up to twelve cells. */
static int tq_neighbors(const orc_geom *g, int64_t key, int l, int64_t *out)
{
    int64_t U, V;
    tq_center_units(g, key, l, &U, &V);
    const int64_t s = (int64_t)1 << (g->L - l);
    const int o = tq_is_up(key, l);
    const int64_t vU[3] = {0, -s, s}, vV[3] = {2 * o * s, -o * s, -o * s};
    const int64_t wU[6] = {0, s, s, 0, -s, -s}, wV[6] = {-2 * s, -s, s, 2 * s, s, -s};
    int cnt = 0;
    for (int v = 0; v < 3; ++v)
        for (int w = 0; w < 6; ++w) {
            int64_t k;
            if (!tq_cell_at(g, U + vU[v] + wU[w], V + vV[v] + wV[w], l, &k) || k == key) continue;
            int dup = 0;
            for (int j = 0; j < cnt; ++j) dup |= (out[j] == k);
            if (!dup) out[cnt++] = k;
        }
    return cnt;
}

/* ===================================================================== */
/* Generic addressing (Sec. 4).                                           */
/* ===================================================================== */

int64_t orc_cell_index(const orc_geom *g, double x, double y, int32_t l)
{
    if (l < 0 || l > g->L) return -1;
    switch (g->tiling) {
    case TIL_QUAD:
        return quad_cell_index(g, x, y, l);
    case TIL_SEPT: {
        int64_t k = sept_leaf_index(g, x, y);
        if (k < 0) return -1;
        return k / ipow(7, g->L - l); /* first l components */
    }
    case TIL_TRI:
        return tq_cell_index(g, x, y, l);
    }
    return -1;
}

void orc_cell_index_many(const orc_geom *g, const double *x, const double *y, int64_t n,
                         int32_t l, int64_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_cell_index(g, x[i], y[i], l);
}

void orc_cell_center(const orc_geom *g, int64_t key, int32_t l, double *cx, double *cy)
{
    switch (g->tiling) {
    case TIL_QUAD:
        quad_center(g, key, l, cx, cy);
        break;
    case TIL_SEPT:
        sept_center(g, key, l, cx, cy);
        break;
    default:
        tq_center(g, key, l, cx, cy);
        break;
    }
}

void orc_cell_center_many(const orc_geom *g, const int64_t *keys, int64_t n, int32_t l,
                          double *cx, double *cy)
{
    for (int64_t i = 0; i < n; ++i) orc_cell_center(g, keys[i], l, cx + i, cy + i);
}

void orc_sept_center_polar(const orc_geom *g, int64_t key, int32_t l, double *cx, double *cy)
{
    sept_center_polar(g, key, l, cx, cy);
}

/* Integer lattice / unit coordinates of a centre (test use). */
void orc_center_units(const orc_geom *g, int64_t key, int32_t l, int64_t *a, int64_t *b)
{
    if (g->tiling == TIL_QUAD) {
        quad_split(key, l, a, b);
    } else if (g->tiling == TIL_SEPT) {
        sept_lattice(g, key, l, a, b);
    } else {
        tq_center_units(g, key, l, a, b);
    }
}

int64_t orc_parent(int32_t tiling, int64_t key) { return key / tiling_base(tiling); }

int32_t orc_neighbors(const orc_geom *g, int64_t key, int32_t l, int64_t *out)
{
    if (l <= 0) return 0;
    switch (g->tiling) {
    case TIL_QUAD:
        return quad_neighbors(key, l, out);
    case TIL_SEPT:
        return sept_neighbors(g, key, l, out);
    default:
        return tq_neighbors(g, key, l, out);
    }
}

/* NeighborsE4(n, l) = Children(Parent(n) u Neighbors(Parent(n), l-1))
 *                     minus ({n} u Neighbors(n, l)).   out needs >= 64. */
int32_t orc_e4(const orc_geom *g, int64_t key, int32_t l, int64_t *out)
{
    if (l < 1) return 0;
    int base = tiling_base(g->tiling);
    int64_t par = key / base;
    int64_t pn[16], own[16];
    int np = orc_neighbors(g, par, l - 1, pn);
    pn[np++] = par;
    int no = orc_neighbors(g, key, l, own);
    own[no++] = key;
    int cnt = 0;
    for (int i = 0; i < np; ++i)
        for (int d = 0; d < base; ++d) {
            int64_t ch = pn[i] * base + d;
            int excluded = 0;
            for (int j = 0; j < no; ++j) excluded |= (own[j] == ch);
            if (!excluded) out[cnt++] = ch;
        }
    return cnt;
}

void orc_e4_many(const orc_geom *g, const int64_t *keys, int64_t n, int32_t l, int64_t *out,
                 int32_t *counts)
{
    for (int64_t i = 0; i < n; ++i) counts[i] = orc_e4(g, keys[i], l, out + 64 * i);
}

void orc_neighbors_many(const orc_geom *g, const int64_t *keys, int64_t n, int32_t l, int64_t *out,
                        int32_t *counts)
{
    for (int64_t i = 0; i < n; ++i) counts[i] = orc_neighbors(g, keys[i], l, out + 16 * i);
}

int64_t orc_gbt_add(int64_t a, int64_t b)
{
    gbt_num x, y;
    gbt_from_key(a, &x);
    gbt_from_key(b, &y);
    if (gbt_add(&x, &y)) return -1;
    return gbt_to_key(&x, 22);
}

/* Edge neighbour of a triangle-quadtree cell (0 = left, 1 = right, 2 =
 * vertical); adjacency does not depend on the placement, so a unit tree of
 * depth l is used. */
int32_t orc_tq_adjacent(int64_t key, int32_t l, int32_t dir, int64_t *out)
{
    if (l < 1 || dir < 0 || dir > 2) return 0;
    orc_geom g = {TIL_TRI, l, 0.0, 0.0, 1.0};
    return tq_adjacent(&g, key, l, dir, out);
}

int32_t orc_tq_is_up(int64_t key, int32_t l) { return tq_is_up(key, l); }

/* ===================================================================== */
/* Expansion and translation operators (Greengard-Rokhlin 1987).          */
/* Coefficients are complex, index 0..p; a multipole expansion about c is */
/*   a_0 log(z - c) + sum_{k=1}^{p} a_k / (z - c)^k,                      */
/* a local expansion about c is sum_{l=0}^{p} b_l (z - c)^l.              */
/* ===================================================================== */

static double *binom_table(int nmax) /* C(n, k) at [n*(nmax+1)+k] */
{
    double *t = calloc((size_t)(nmax + 1) * (nmax + 1), sizeof(double));
    for (int n = 0; n <= nmax; ++n) {
        t[n * (nmax + 1)] = 1.0;
        for (int k = 1; k <= n; ++k)
            t[n * (nmax + 1) + k] = t[(n - 1) * (nmax + 1) + k - 1] +
                                    (k <= n - 1 ? t[(n - 1) * (nmax + 1) + k] : 0.0);
    }
    return t;
}
#define BIN(tab, nmax, n, k) ((tab)[(n) * ((nmax) + 1) + (k)])

/* Lemma 2.1: a_0 = sum u_i, a_k = -sum u_i (x_i - c)^k / k. */
static void op_p2m(int p, cplx c, int64_t n, const int64_t *idx, const double *xs, const double *ys,
                   const double *u, cplx *a)
{
    for (int64_t m = 0; m < n; ++m) {
        int64_t i = idx ? idx[m] : m;
        cplx w = CMPLX(xs[i], ys[i]) - c;
        a[0] += u[i];
        cplx pw = 1.0;
        for (int k = 1; k <= p; ++k) {
            pw *= w;
            a[k] -= u[i] * pw / (double)k;
        }
    }
}

/* Lemma 2.3: shift a multipole about c_child by z0 = c_child - c_parent. */
static void op_m2m(int p, const cplx *a, cplx z0, const double *bt, int nmax, cplx *b)
{
    cplx zp[128];
    zp[0] = 1.0;
    for (int i = 1; i <= p; ++i) zp[i] = zp[i - 1] * z0;
    b[0] += a[0];
    for (int l = 1; l <= p; ++l) {
        cplx s = -a[0] * zp[l] / (double)l;
        for (int k = 1; k <= l; ++k) s += a[k] * zp[l - k] * BIN(bt, nmax, l - 1, k - 1);
        b[l] += s;
    }
}

/* Lemma 2.4: multipole about c_S to local about c_T, z0 = c_S - c_T,
 * log term Log(c_T - c_S). */
static void op_m2l(int p, const cplx *a, cplx cS, cplx cT, const double *bt, int nmax, cplx *b)
{
    cplx z0 = cS - cT;
    cplx lg = log_canon(cT - cS);
    cplx iz = 1.0 / z0;
    cplx izp[128];
    izp[0] = 1.0;
    for (int i = 1; i <= 2 * p + 1 && i < 128; ++i) izp[i] = izp[i - 1] * iz;
    cplx s0 = a[0] * lg;
    for (int k = 1; k <= p; ++k) s0 += ((k & 1) ? -1.0 : 1.0) * a[k] * izp[k];
    b[0] += s0;
    for (int l = 1; l <= p; ++l) {
        cplx s = 0.0;
        for (int k = 1; k <= p; ++k)
            s += ((k & 1) ? -1.0 : 1.0) * a[k] * izp[k] * BIN(bt, nmax, l + k - 1, k - 1);
        b[l] += -a[0] * izp[l] / (double)l + izp[l] * s;
    }
}

/* Lemma 2.5: local about c_parent to local about c_child, w = c_child - c_parent. */
static void op_l2l(int p, const cplx *b, cplx w, const double *bt, int nmax, cplx *out)
{
    cplx wp[128];
    wp[0] = 1.0;
    for (int i = 1; i <= p; ++i) wp[i] = wp[i - 1] * w;
    for (int l = 0; l <= p; ++l) {
        cplx s = 0.0;
        for (int k = l; k <= p; ++k) s += b[k] * BIN(bt, nmax, k, l) * wp[k - l];
        out[l] += s;
    }
}

static cplx op_l2p(int p, const cplx *b, cplx c, cplx y)
{
    cplx w = y - c, pw = 1.0, s = 0.0;
    for (int l = 0; l <= p; ++l) {
        s += b[l] * pw;
        pw *= w;
    }
    return s;
}

/* Derivative of the local expansion at y: sum_{l>=1} l b_l (y - c)^(l-1)
 * (the field output, d/dy of the L2P sum). */
static cplx op_l2p_deriv(int p, const cplx *b, cplx c, cplx y)
{
    cplx w = y - c, pw = 1.0, s = 0.0;
    for (int l = 1; l <= p; ++l) {
        s += (double)l * b[l] * pw;
        pw *= w;
    }
    return s;
}

/* Evaluate a multipole expansion at a point (test use). */
static cplx op_mpole_eval(int p, const cplx *a, cplx c, cplx y)
{
    cplx w = y - c;
    cplx s = a[0] * log_canon(w);
    cplx iw = 1.0 / w, pw = 1.0;
    for (int k = 1; k <= p; ++k) {
        pw *= iw;
        s += a[k] * pw;
    }
    return s;
}

/* Exported single-operator entry points; coefficient arrays are interleaved
 * (re, im) doubles of length 2(p+1).  Outputs accumulate. */
void orc_op_p2m(int32_t p, double cx, double cy, int64_t n, const double *x, const double *y,
                const double *u, double *a)
{
    op_p2m(p, CMPLX(cx, cy), n, NULL, x, y, u, (cplx *)a);
}

void orc_op_m2m(int32_t p, const double *a, double z0x, double z0y, double *b)
{
    double *bt = binom_table(2 * p + 2);
    op_m2m(p, (const cplx *)a, CMPLX(z0x, z0y), bt, 2 * p + 2, (cplx *)b);
    free(bt);
}

void orc_op_m2l(int32_t p, const double *a, double csx, double csy, double ctx, double cty, double *b)
{
    double *bt = binom_table(2 * p + 2);
    op_m2l(p, (const cplx *)a, CMPLX(csx, csy), CMPLX(ctx, cty), bt, 2 * p + 2, (cplx *)b);
    free(bt);
}

void orc_op_l2l(int32_t p, const double *b, double wx, double wy, double *out)
{
    double *bt = binom_table(2 * p + 2);
    op_l2l(p, (const cplx *)b, CMPLX(wx, wy), bt, 2 * p + 2, (cplx *)out);
    free(bt);
}

void orc_op_l2p(int32_t p, const double *b, double cx, double cy, int64_t n, const double *x,
                const double *y, double *phi)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx v = op_l2p(p, (const cplx *)b, CMPLX(cx, cy), CMPLX(x[i], y[i]));
        phi[2 * i] += creal(v);
        phi[2 * i + 1] += cimag(v);
    }
}

void orc_op_mpole_eval(int32_t p, const double *a, double cx, double cy, int64_t n, const double *x,
                       const double *y, double *phi)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx v = op_mpole_eval(p, (const cplx *)a, CMPLX(cx, cy), CMPLX(x[i], y[i]));
        phi[2 * i] += creal(v);
        phi[2 * i + 1] += cimag(v);
    }
}

/* ===================================================================== */
/* Direct sums.                                                           */
/* ===================================================================== */

/* Neumaier compensated accumulation. */
typedef struct { double s, c; } nsum;
static void nadd(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static void set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* D1: principal direct sum, coincident pairs skipped. */
void orc_direct_principal(int64_t ns, const double *xs, const double *ys, const double *u,
                          int64_t nt, const double *xt, const double *yt, double *phi,
                          int32_t nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nt; ++j) {
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t i = 0; i < ns; ++i) {
            if (xs[i] == xt[j] && ys[i] == yt[j]) continue;
            cplx lg = log_canon(CMPLX(xt[j] - xs[i], yt[j] - ys[i]));
            nadd(&re, u[i] * creal(lg));
            nadd(&im, u[i] * cimag(lg));
        }
        phi[2 * j] = re.s + re.c;
        phi[2 * j + 1] = im.s + im.c;
    }
}

/* Field Phi'(y_j) = sum_i u_i / (y_j - x_i) (the derivative of eq. 2 in
 * y), coincident pairs skipped, compensated sums. */
void orc_direct_field(int64_t ns, const double *xs, const double *ys, const double *u, int64_t nt,
                      const double *xt, const double *yt, double *out, int32_t nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t j = 0; j < nt; ++j) {
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t i = 0; i < ns; ++i) {
            if (xs[i] == xt[j] && ys[i] == yt[j]) continue;
            cplx q = u[i] / CMPLX(xt[j] - xs[i], yt[j] - ys[i]);
            nadd(&re, creal(q));
            nadd(&im, cimag(q));
        }
        out[2 * j] = re.s + re.c;
        out[2 * j + 1] = im.s + im.c;
    }
}

static int64_t level_key(int tiling, int L, int64_t leaf, int l)
{
    if (tiling == TIL_SEPT) return leaf / ipow(7, L - l);
    return leaf >> (2 * (L - l));
}

static int in_closed_nbhd(const orc_geom *g, int64_t a, int64_t b, int l) /* a in {b} u Nbrs(b) */
{
    if (a == b) return 1;
    int64_t nb[16];
    int n = orc_neighbors(g, b, l, nb);
    for (int i = 0; i < n; ++i)
        if (nb[i] == a) return 1;
    return 0;
}

/* Level at which leaf pair (source leaf s, target leaf t) is handled:
 * 0 = near field at the leaf level, l >= 1 = E4 at level l, -1 = neither. */
static int pair_level(const orc_geom *g, int64_t s, int64_t t)
{
    int L = g->L;
    if (in_closed_nbhd(g, s, t, L)) return 0;
    /* Walking up, the cells stay separated until their parents touch. */
    for (int l = L; l >= 1; --l) {
        int64_t sp = level_key(g->tiling, L, s, l - 1), tp = level_key(g->tiling, L, t, l - 1);
        if (in_closed_nbhd(g, sp, tp, l - 1)) return l;
    }
    return -1;
}

/* D2: branch-aware direct sum.  Far pairs use
 *   Log(c_T - c_S) + Log((y - x) / (c_T - c_S))
 * with (S, T) the unique E4 cell pair that separates them; near pairs use
 * Log(y - x).  Returns 0, or 2 if a point lies outside the root. */
int32_t orc_direct_branch_aware(const orc_geom *g, int64_t ns, const double *xs, const double *ys,
                                const double *u, int64_t nt, const double *xt, const double *yt,
                                double *phi, int32_t nthreads)
{
    int L = g->L;
    int64_t *ks = malloc(sizeof(int64_t) * (ns > 0 ? ns : 1));
    int64_t *kt = malloc(sizeof(int64_t) * (nt > 0 ? nt : 1));
    for (int64_t i = 0; i < ns; ++i) {
        ks[i] = orc_cell_index(g, xs[i], ys[i], L);
        if (ks[i] < 0) {
            free(ks);
            free(kt);
            return 2;
        }
    }
    for (int64_t j = 0; j < nt; ++j) {
        kt[j] = orc_cell_index(g, xt[j], yt[j], L);
        if (kt[j] < 0) {
            free(ks);
            free(kt);
            return 2;
        }
    }
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t j = 0; j < nt; ++j) {
        nsum re = {0, 0}, im = {0, 0};
        int64_t last_s = -1;
        int lev = 0;
        for (int64_t i = 0; i < ns; ++i) {
            if (xs[i] == xt[j] && ys[i] == yt[j]) continue;
            if (ks[i] != last_s) {
                lev = pair_level(g, ks[i], kt[j]);
                last_s = ks[i];
            }
            cplx d = CMPLX(xt[j] - xs[i], yt[j] - ys[i]);
            cplx lg;
            if (lev <= 0) {
                lg = log_canon(d);
            } else {
                double csx, csy, ctx, cty;
                orc_cell_center(g, level_key(g->tiling, L, ks[i], lev), lev, &csx, &csy);
                orc_cell_center(g, level_key(g->tiling, L, kt[j], lev), lev, &ctx, &cty);
                cplx dc = CMPLX(ctx - csx, cty - csy);
                lg = log_canon(dc) + log_canon(d / dc);
            }
            nadd(&re, u[i] * creal(lg));
            nadd(&im, u[i] * cimag(lg));
        }
        phi[2 * j] = re.s + re.c;
        phi[2 * j + 1] = im.s + im.c;
    }
    free(ks);
    free(kt);
    return 0;
}

/* ===================================================================== */
/* The FMM sweep.                                                         */
/* ===================================================================== */

typedef struct { int64_t key, idx; } kidx;

static int cmp_kidx(const void *a, const void *b)
{
    const kidx *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

typedef struct {
    int64_t n;
    int64_t *key;   /* sorted cell keys at this level */
    int64_t *begin; /* range into the sorted point order */
    int64_t *end;
} cells;

static void build_cells(const kidx *pts, int64_t np, int tiling, int L, int l, cells *c)
{
    c->n = 0;
    c->key = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
    c->begin = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
    c->end = malloc(sizeof(int64_t) * (np > 0 ? np : 1));
    for (int64_t i = 0; i < np; ++i) {
        int64_t k = level_key(tiling, L, pts[i].key, l);
        if (c->n == 0 || c->key[c->n - 1] != k) {
            c->key[c->n] = k;
            c->begin[c->n] = i;
            c->n++;
        }
        c->end[c->n - 1] = i + 1;
    }
}

static void free_cells(cells *c)
{
    free(c->key);
    free(c->begin);
    free(c->end);
}

static int64_t find_cell(const cells *c, int64_t key)
{
    int64_t lo = 0, hi = c->n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (c->key[mid] == key) return mid;
        if (c->key[mid] < key)
            lo = mid + 1;
        else
            hi = mid - 1;
    }
    return -1;
}

/* Full FMM: keys, tree, P2M, M2M, M2L, L2L, L2P + P2P.  phi is 2*nt
 * interleaved (re, im) in the caller's target order.  times (optional, 6
 * doubles) receives the wall time of: keys+tree, P2M+M2M, M2L, L2L,
 * L2P+P2P, total.  Returns 0, 1 on bad arguments, 2 if a point lies
 * outside the root. */
static int32_t fmm_run(const orc_geom *g, int32_t p, int64_t ns, const double *xs, const double *ys,
                       const double *u, int64_t nt, const double *xt, const double *yt, double *phi,
                       double *field, int32_t nthreads, double *times)
{
    if (p < 1 || p > 60 || g->L < 0 || ns < 0 || nt < 0) return 1;
    set_threads(nthreads);
    const int L = g->L, tiling = g->tiling, base = tiling_base(tiling);
    const int nmax = 2 * p + 2;
    double t0 = now_s();
    double *bt = binom_table(nmax);

    kidx *sk = malloc(sizeof(kidx) * (ns > 0 ? ns : 1));
    kidx *tk = malloc(sizeof(kidx) * (nt > 0 ? nt : 1));
    int bad = 0;
    for (int64_t i = 0; i < ns; ++i) {
        sk[i].key = orc_cell_index(g, xs[i], ys[i], L);
        sk[i].idx = i;
        bad |= sk[i].key < 0;
    }
    for (int64_t j = 0; j < nt; ++j) {
        tk[j].key = orc_cell_index(g, xt[j], yt[j], L);
        tk[j].idx = j;
        bad |= tk[j].key < 0;
    }
    if (bad) {
        free(sk);
        free(tk);
        free(bt);
        return 2;
    }
    qsort(sk, (size_t)ns, sizeof(kidx), cmp_kidx);
    qsort(tk, (size_t)nt, sizeof(kidx), cmp_kidx);
    int64_t *sidx = malloc(sizeof(int64_t) * (ns > 0 ? ns : 1));
    for (int64_t i = 0; i < ns; ++i) sidx[i] = sk[i].idx;

    cells *sc = calloc((size_t)L + 1, sizeof(cells));
    cells *tc = calloc((size_t)L + 1, sizeof(cells));
    for (int l = 0; l <= L; ++l) {
        build_cells(sk, ns, tiling, L, l, &sc[l]);
        build_cells(tk, nt, tiling, L, l, &tc[l]);
    }
    const int P1 = p + 1;
    cplx **mp = calloc((size_t)L + 1, sizeof(cplx *));
    cplx **lc = calloc((size_t)L + 1, sizeof(cplx *));
    for (int l = 0; l <= L; ++l) {
        mp[l] = calloc((size_t)(sc[l].n > 0 ? sc[l].n : 1) * P1, sizeof(cplx));
        lc[l] = calloc((size_t)(tc[l].n > 0 ? tc[l].n : 1) * P1, sizeof(cplx));
    }
    double t1 = now_s();

    /* P2M at the leaves. */
    for (int64_t c = 0; c < sc[L].n; ++c) {
        double cx, cy;
        orc_cell_center(g, sc[L].key[c], L, &cx, &cy);
        op_p2m(p, CMPLX(cx, cy), sc[L].end[c] - sc[L].begin[c], sidx + sc[L].begin[c], xs, ys, u,
               mp[L] + c * P1);
    }
    /* M2M, finest to coarsest. */
    for (int l = L - 1; l >= 0; --l) {
        for (int64_t c = 0; c < sc[l].n; ++c) {
            double px, py;
            orc_cell_center(g, sc[l].key[c], l, &px, &py);
            for (int d = 0; d < base; ++d) {
                int64_t ch = find_cell(&sc[l + 1], sc[l].key[c] * base + d);
                if (ch < 0) continue;
                double cx, cy;
                orc_cell_center(g, sc[l + 1].key[ch], l + 1, &cx, &cy);
                op_m2m(p, mp[l + 1] + ch * P1, CMPLX(cx - px, cy - py), bt, nmax, mp[l] + c * P1);
            }
        }
    }
    double t2 = now_s();

    /* M2L over each level's interaction lists. */
    for (int l = 1; l <= L; ++l) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t c = 0; c < tc[l].n; ++c) {
            int64_t e4[64];
            int ne = orc_e4(g, tc[l].key[c], l, e4);
            double ctx, cty;
            orc_cell_center(g, tc[l].key[c], l, &ctx, &cty);
            for (int e = 0; e < ne; ++e) {
                int64_t s = find_cell(&sc[l], e4[e]);
                if (s < 0) continue;
                double csx, csy;
                orc_cell_center(g, e4[e], l, &csx, &csy);
                op_m2l(p, mp[l] + s * P1, CMPLX(csx, csy), CMPLX(ctx, cty), bt, nmax,
                       lc[l] + c * P1);
            }
        }
    }
    double t3 = now_s();

    /* L2L, coarsest to finest. */
    for (int l = 1; l < L; ++l) {
        for (int64_t c = 0; c < tc[l + 1].n; ++c) {
            int64_t par = find_cell(&tc[l], tc[l + 1].key[c] / base);
            double px, py, cx, cy;
            orc_cell_center(g, tc[l].key[par], l, &px, &py);
            orc_cell_center(g, tc[l + 1].key[c], l + 1, &cx, &cy);
            op_l2l(p, lc[l] + par * P1, CMPLX(cx - px, cy - py), bt, nmax, lc[l + 1] + c * P1);
        }
    }
    double t4 = now_s();

    /* L2P and P2P per target leaf. */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t c = 0; c < tc[L].n; ++c) {
        int64_t tkey = tc[L].key[c];
        double cx, cy;
        orc_cell_center(g, tkey, L, &cx, &cy);
        int64_t nb[16];
        int nn = orc_neighbors(g, tkey, L, nb);
        nb[nn++] = tkey;
        for (int64_t m = tc[L].begin[c]; m < tc[L].end[c]; ++m) {
            int64_t j = tk[m].idx;
            cplx y = CMPLX(xt[j], yt[j]);
            cplx far = op_l2p(p, lc[L] + c * P1, CMPLX(cx, cy), y);
            nsum re = {0, 0}, im = {0, 0}, fre = {0, 0}, fim = {0, 0};
            for (int q = 0; q < nn; ++q) {
                int64_t s = find_cell(&sc[L], nb[q]);
                if (s < 0) continue;
                for (int64_t a = sc[L].begin[s]; a < sc[L].end[s]; ++a) {
                    int64_t i = sidx[a];
                    if (xs[i] == xt[j] && ys[i] == yt[j]) continue;
                    cplx lg = log_canon(CMPLX(xt[j] - xs[i], yt[j] - ys[i]));
                    nadd(&re, u[i] * creal(lg));
                    nadd(&im, u[i] * cimag(lg));
                    if (field) {
                        cplx fq = u[i] / CMPLX(xt[j] - xs[i], yt[j] - ys[i]);
                        nadd(&fre, creal(fq));
                        nadd(&fim, cimag(fq));
                    }
                }
            }
            phi[2 * j] = creal(far) + (re.s + re.c);
            phi[2 * j + 1] = cimag(far) + (im.s + im.c);
            if (field) {
                cplx fd = op_l2p_deriv(p, lc[L] + c * P1, CMPLX(cx, cy), y);
                field[2 * j] = creal(fd) + (fre.s + fre.c);
                field[2 * j + 1] = cimag(fd) + (fim.s + fim.c);
            }
        }
    }
    double t5 = now_s();
    if (times) {
        times[0] = t1 - t0;
        times[1] = t2 - t1;
        times[2] = t3 - t2;
        times[3] = t4 - t3;
        times[4] = t5 - t4;
        times[5] = t5 - t0;
    }

    for (int l = 0; l <= L; ++l) {
        free(mp[l]);
        free(lc[l]);
        free_cells(&sc[l]);
        free_cells(&tc[l]);
    }
    free(mp);
    free(lc);
    free(sc);
    free(tc);
    free(sk);
    free(tk);
    free(sidx);
    free(bt);
    return 0;
}

int32_t orc_fmm(const orc_geom *g, int32_t p, int64_t ns, const double *xs, const double *ys,
                const double *u, int64_t nt, const double *xt, const double *yt, double *phi,
                int32_t nthreads, double *times)
{
    return fmm_run(g, p, ns, xs, ys, u, nt, xt, yt, phi, NULL, nthreads, times);
}

/* As orc_fmm, and the field Phi'(y_j) (2*nt interleaved, caller's order):
 * the derivative of the leaf's local expansion plus sum u_i / (y_j - x_i)
 * over the same near sources. */
int32_t orc_fmm_field(const orc_geom *g, int32_t p, int64_t ns, const double *xs, const double *ys,
                      const double *u, int64_t nt, const double *xt, const double *yt, double *phi,
                      double *field, int32_t nthreads, double *times)
{
    return fmm_run(g, p, ns, xs, ys, u, nt, xt, yt, phi, field, nthreads, times);
}

/* Multipole coefficients of every source-occupied cell at level l after the
 * upward pass (test use: the monopole invariant and M2M exactness).
 * keys_out / coef_out must hold the number of source cells at level l;
 * call with coef_out == NULL to get the count. */
int64_t orc_upward_level(const orc_geom *g, int32_t p, int64_t ns, const double *xs,
                         const double *ys, const double *u, int32_t level, int64_t *keys_out,
                         double *coef_out)
{
    const int L = g->L, tiling = g->tiling, base = tiling_base(tiling), nmax = 2 * p + 2;
    if (level < 0 || level > L) return -1;
    kidx *sk = malloc(sizeof(kidx) * (ns > 0 ? ns : 1));
    for (int64_t i = 0; i < ns; ++i) {
        sk[i].key = orc_cell_index(g, xs[i], ys[i], L);
        sk[i].idx = i;
        if (sk[i].key < 0) {
            free(sk);
            return -2;
        }
    }
    qsort(sk, (size_t)ns, sizeof(kidx), cmp_kidx);
    int64_t *sidx = malloc(sizeof(int64_t) * (ns > 0 ? ns : 1));
    for (int64_t i = 0; i < ns; ++i) sidx[i] = sk[i].idx;
    cells *sc = calloc((size_t)L + 1, sizeof(cells));
    for (int l = 0; l <= L; ++l) build_cells(sk, ns, tiling, L, l, &sc[l]);
    int64_t count = sc[level].n;
    if (coef_out) {
        double *bt = binom_table(nmax);
        const int P1 = p + 1;
        cplx **mp = calloc((size_t)L + 1, sizeof(cplx *));
        for (int l = 0; l <= L; ++l) mp[l] = calloc((size_t)(sc[l].n > 0 ? sc[l].n : 1) * P1, sizeof(cplx));
        for (int64_t c = 0; c < sc[L].n; ++c) {
            double cx, cy;
            orc_cell_center(g, sc[L].key[c], L, &cx, &cy);
            op_p2m(p, CMPLX(cx, cy), sc[L].end[c] - sc[L].begin[c], sidx + sc[L].begin[c], xs, ys,
                   u, mp[L] + c * P1);
        }
        for (int l = L - 1; l >= level; --l)
            for (int64_t c = 0; c < sc[l].n; ++c) {
                double px, py;
                orc_cell_center(g, sc[l].key[c], l, &px, &py);
                for (int d = 0; d < base; ++d) {
                    int64_t ch = find_cell(&sc[l + 1], sc[l].key[c] * base + d);
                    if (ch < 0) continue;
                    double cx, cy;
                    orc_cell_center(g, sc[l + 1].key[ch], l + 1, &cx, &cy);
                    op_m2m(p, mp[l + 1] + ch * P1, CMPLX(cx - px, cy - py), bt, nmax,
                           mp[l] + c * P1);
                }
            }
        for (int64_t c = 0; c < count; ++c) {
            keys_out[c] = sc[level].key[c];
            for (int k = 0; k <= p; ++k) {
                coef_out[2 * (c * P1 + k)] = creal(mp[level][c * P1 + k]);
                coef_out[2 * (c * P1 + k) + 1] = cimag(mp[level][c * P1 + k]);
            }
        }
        for (int l = 0; l <= L; ++l) free(mp[l]);
        free(mp);
        free(bt);
    }
    for (int l = 0; l <= L; ++l) free_cells(&sc[l]);
    free(sc);
    free(sk);
    free(sidx);
    return count;
}
