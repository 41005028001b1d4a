/*
 * sd3 oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow FP64 CPU reference for the two spatial operators of
 * "Full Speed Ahead: 3D Spatial Database Acceleration with GPUs" (arXiv
 * 1808.09571): the 3D distance and the 3D intersection test between two
 * triangulated surfaces (TINs / polyhedral surfaces).  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load this library; the
 * GPU library never links or calls it, and the two share no code.
 *
 * What is computed (Sec. 3.2.2 "Distance", Sec. 3.2.3 "Intersection"):
 *   A surface is the union of its closed triangles.  The distance is the
 *   minimum, over every pair (triangle of A, triangle of B), of the distance
 *   between the two closed triangles (the per-face distances of Sec. 3.2.2
 *   followed by the minimum that is returned to the user).  Intersects is true
 *   iff some pair of closed triangles shares a point (the per-face tests of
 *   Sec. 3.2.3, all constraints taken as closed, i.e. touching counts).
 *   The distance is 0 iff the surfaces intersect; +inf if either is empty.
 *
 * Triangle-pair distance.  For two disjoint closed triangles a closest pair of
 * points has at least one point on the boundary of its triangle, so the
 * distance is the minimum of the 9 edge/edge distances (Sec. 3.2.2 item (i),
 * segment/segment) and the 6 vertex/face distances (item (iii),
 * point/surface).  The edge/edge distance minimises the convex quadratic
 * Q(s,t) = |P(s) - Q(t)|^2 over the closed unit square (the squared-distance
 * minimisation of Eq. 3, with a segment in place of the triangle): the
 * minimum is either the interior stationary point or lies on one of the four
 * sides, each a clamped point/segment projection.
 *
 * Intersection.  Two closed triangles meet iff an edge of one meets the other
 * closed triangle.  A segment meets a closed triangle iff its end points are
 * not strictly on the same side of the triangle's plane and the line through
 * it passes through the triangle -- the segment/plane/barycentric test of
 * Eq. 4 (t in [0,1], u, v >= 0, u + v <= 1), with every division replaced by
 * the sign of the corresponding determinant so that the answer is exact.
 * Coplanar and degenerate configurations are decided exactly in 2D.
 *
 * Exactness.  orient3d/orient2d are evaluated in FP64 with a forward error
 * bound; when the bound cannot decide the sign, the determinant is recomputed
 * exactly with arbitrary-precision integers (every double is an integer times a
 * power of two).  This requires every nonzero |coordinate| to lie in
 * [2^-256, 2^256] so that no product underflows or overflows; the wrapper
 * checks that.
 *
 * Numerics of the distance: all vectors between the two triangles are formed
 * by subtracting input coordinates first (p - q), then combined, so rounding
 * error scales with the local extent rather than with the absolute
 * coordinates.  Built with -ffp-contract=off, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------------- */
/* Exact signs through arbitrary-precision integers                            */
/* ------------------------------------------------------------------------- */
#define BN_N 72 /* 2304 bits: a product of three 566-bit differences fits */

typedef struct {
    int neg;
    int n; /* used limbs; 0 means zero */
    uint32_t d[BN_N];
} bn;

static long long g_exact_calls;

static void bn_norm(bn *a) {
    while (a->n > 0 && a->d[a->n - 1] == 0) a->n--;
    if (a->n == 0) a->neg = 0;
}

/* exponent of the last bit of x: x = m * 2^ulp_exp(x) with m an integer */
static int ulp_exp(double x) {
    int e;
    frexp(x, &e);
    return e - 53;
}

/* r = x / 2^e0 exactly (x must be a multiple of 2^e0) */
static void bn_from_double(bn *r, double x, int e0) {
    memset(r, 0, sizeof *r);
    if (x == 0.0) return;
    int e;
    double f = frexp(fabs(x), &e);
    uint64_t m = (uint64_t)ldexp(f, 53);
    int sh = e - 53 - e0;
    int limb = sh / 32, bit = sh % 32;
    unsigned __int128 v = (unsigned __int128)m << bit;
    r->d[limb] = (uint32_t)v;
    r->d[limb + 1] = (uint32_t)(v >> 32);
    r->d[limb + 2] = (uint32_t)(v >> 64);
    r->n = limb + 3;
    r->neg = x < 0.0;
    bn_norm(r);
}

static int bn_cmp_mag(const bn *a, const bn *b) {
    if (a->n != b->n) return a->n < b->n ? -1 : 1;
    for (int i = a->n - 1; i >= 0; i--)
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    return 0;
}

/* |r| = |a| + |b| */
static void bn_add_mag(bn *r, const bn *a, const bn *b) {
    int n = a->n > b->n ? a->n : b->n;
    uint64_t c = 0;
    for (int i = 0; i < n; i++) {
        uint64_t s = c;
        if (i < a->n) s += a->d[i];
        if (i < b->n) s += b->d[i];
        r->d[i] = (uint32_t)s;
        c = s >> 32;
    }
    r->d[n] = (uint32_t)c;
    r->n = n + 1;
}

/* |r| = |a| - |b|, requires |a| >= |b| */
static void bn_sub_mag(bn *r, const bn *a, const bn *b) {
    int64_t br = 0;
    for (int i = 0; i < a->n; i++) {
        int64_t s = (int64_t)a->d[i] - br - (i < b->n ? (int64_t)b->d[i] : 0);
        br = s < 0;
        if (s < 0) s += ((int64_t)1 << 32);
        r->d[i] = (uint32_t)s;
    }
    r->n = a->n;
}

static void bn_add(bn *r, const bn *a, const bn *b) {
    bn t;
    memset(&t, 0, sizeof t);
    if (a->neg == b->neg) {
        bn_add_mag(&t, a, b);
        t.neg = a->neg;
    } else if (bn_cmp_mag(a, b) >= 0) {
        bn_sub_mag(&t, a, b);
        t.neg = a->neg;
    } else {
        bn_sub_mag(&t, b, a);
        t.neg = b->neg;
    }
    bn_norm(&t);
    *r = t;
}

static void bn_sub(bn *r, const bn *a, const bn *b) {
    bn nb = *b;
    if (nb.n) nb.neg = !nb.neg;
    bn_add(r, a, &nb);
}

static void bn_mul(bn *r, const bn *a, const bn *b) {
    bn t;
    memset(&t, 0, sizeof t);
    if (a->n == 0 || b->n == 0) {
        *r = t;
        return;
    }
    if (a->n + b->n > BN_N) abort(); /* inputs outside the documented range */
    for (int i = 0; i < a->n; i++) {
        uint64_t c = 0;
        for (int j = 0; j < b->n; j++) {
            uint64_t s = (uint64_t)a->d[i] * b->d[j] + t.d[i + j] + c;
            t.d[i + j] = (uint32_t)s;
            c = s >> 32;
        }
        t.d[i + b->n] = (uint32_t)c;
    }
    t.n = a->n + b->n;
    t.neg = a->neg != b->neg;
    bn_norm(&t);
    *r = t;
}

static int bn_sign(const bn *a) { return a->n == 0 ? 0 : (a->neg ? -1 : 1); }

static int min_ulp_exp(const double *v, int k) {
    int e0 = 1 << 20;
    for (int i = 0; i < k; i++)
        if (v[i] != 0.0) {
            int e = ulp_exp(v[i]);
            if (e < e0) e0 = e;
        }
    return e0 == (1 << 20) ? 0 : e0;
}

/* sign of det[b-a, c-a, d-a], exactly */
int sd3o_orient3d_exact(const double *a, const double *b, const double *c, const double *d) {
    __atomic_fetch_add(&g_exact_calls, 1, __ATOMIC_RELAXED);
    double all[12] = {a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2], d[0], d[1], d[2]};
    int e0 = min_ulp_exp(all, 12);
    bn A[3], B[3], C[3], D[3], u[3], v[3], w[3];
    for (int i = 0; i < 3; i++) {
        bn_from_double(&A[i], a[i], e0);
        bn_from_double(&B[i], b[i], e0);
        bn_from_double(&C[i], c[i], e0);
        bn_from_double(&D[i], d[i], e0);
        bn_sub(&u[i], &B[i], &A[i]);
        bn_sub(&v[i], &C[i], &A[i]);
        bn_sub(&w[i], &D[i], &A[i]);
    }
    /* (u x v) . w */
    bn det, t1, t2, m, p;
    memset(&det, 0, sizeof det);
    for (int i = 0; i < 3; i++) {
        int j = (i + 1) % 3, k = (i + 2) % 3;
        bn_mul(&t1, &u[j], &v[k]);
        bn_mul(&t2, &u[k], &v[j]);
        bn_sub(&m, &t1, &t2);
        bn_mul(&p, &m, &w[i]);
        bn_add(&det, &det, &p);
    }
    return bn_sign(&det);
}

/* sign of (b-a) x (c-a) in 2D, exactly */
int sd3o_orient2d_exact(const double *a, const double *b, const double *c) {
    __atomic_fetch_add(&g_exact_calls, 1, __ATOMIC_RELAXED);
    double all[6] = {a[0], a[1], b[0], b[1], c[0], c[1]};
    int e0 = min_ulp_exp(all, 6);
    bn A[2], B[2], C[2], u[2], v[2], t1, t2, det;
    for (int i = 0; i < 2; i++) {
        bn_from_double(&A[i], a[i], e0);
        bn_from_double(&B[i], b[i], e0);
        bn_from_double(&C[i], c[i], e0);
        bn_sub(&u[i], &B[i], &A[i]);
        bn_sub(&v[i], &C[i], &A[i]);
    }
    bn_mul(&t1, &u[0], &v[1]);
    bn_mul(&t2, &u[1], &v[0]);
    bn_sub(&det, &t1, &t2);
    return bn_sign(&det);
}

long long sd3o_exact_calls(void) { return __atomic_load_n(&g_exact_calls, __ATOMIC_RELAXED); }

/* ------------------------------------------------------------------------- */
/* Filtered predicates                                                         */
/* ------------------------------------------------------------------------- */
/*
 * orient3d(a,b,c,d) = ((b-a) x (c-a)) . (d-a); > 0 when d lies on the side the
 * normal (b-a) x (c-a) points to.
 *
 * FP64 error bound (u = 2^-53, no underflow/overflow): each of the 6
 * elementary triple products of the expansion passes through at most 8
 * roundings (3 differences, 1 product, 1 minor subtraction, 1 product, 2
 * additions), so |computed - exact| <= ((1+u)^8 - 1) * P with P the sum of
 * the absolute triple products; the P computed in floating point is at least
 * (1-u)^8 times the exact one.  Hence 9u * P_computed bounds the error and a
 * larger |computed| has the right sign.
 */
static const double U64 = 1.1102230246251565e-16; /* 2^-53 */

int sd3o_orient3d(const double *a, const double *b, const double *c, const double *d) {
    double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
    double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
    double wx = d[0] - a[0], wy = d[1] - a[1], wz = d[2] - a[2];
    double mx = uy * vz - uz * vy;
    double my = uz * vx - ux * vz;
    double mz = ux * vy - uy * vx;
    double det = mx * wx + my * wy + mz * wz;
    double perm = (fabs(uy * vz) + fabs(uz * vy)) * fabs(wx) +
                  (fabs(uz * vx) + fabs(ux * vz)) * fabs(wy) +
                  (fabs(ux * vy) + fabs(uy * vx)) * fabs(wz);
    double bound = 9.0 * U64 * perm;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    if (perm == 0.0) return 0;
    return sd3o_orient3d_exact(a, b, c, d);
}

/* 2D: 4 roundings per elementary product (2 differences, product,
 * subtraction); 5u * P_computed bounds the error. */
int sd3o_orient2d(const double *a, const double *b, const double *c) {
    double ux = b[0] - a[0], uy = b[1] - a[1];
    double vx = c[0] - a[0], vy = c[1] - a[1];
    double det = ux * vy - uy * vx;
    double perm = fabs(ux * vy) + fabs(uy * vx);
    double bound = 5.0 * U64 * perm;
    if (det > bound) return 1;
    if (-det > bound) return -1;
    if (perm == 0.0) return 0;
    return sd3o_orient2d_exact(a, b, c);
}

/* ------------------------------------------------------------------------- */
/* Exact intersection of closed segments and triangles                        */
/* ------------------------------------------------------------------------- */
/* drop coordinate k */
static void proj(const double *p, int k, double out[2]) {
    out[0] = p[(k + 1) % 3];
    out[1] = p[(k + 2) % 3];
}

/* r on the closed segment [p, q], given that the three are collinear */
static int in_box2(const double *p, const double *q, const double *r) {
    for (int i = 0; i < 2; i++) {
        double lo = p[i] < q[i] ? p[i] : q[i];
        double hi = p[i] < q[i] ? q[i] : p[i];
        if (r[i] < lo || r[i] > hi) return 0;
    }
    return 1;
}

/* closed 2D segments [p,q] and [r,s] share a point */
static int seg_seg_2d(const double *p, const double *q, const double *r, const double *s) {
    int o1 = sd3o_orient2d(p, q, r), o2 = sd3o_orient2d(p, q, s);
    int o3 = sd3o_orient2d(r, s, p), o4 = sd3o_orient2d(r, s, q);
    if (o1 * o2 < 0 && o3 * o4 < 0) return 1;
    if (o1 == 0 && in_box2(p, q, r)) return 1;
    if (o2 == 0 && in_box2(p, q, s)) return 1;
    if (o3 == 0 && in_box2(r, s, p)) return 1;
    if (o4 == 0 && in_box2(r, s, q)) return 1;
    return 0;
}

/* closed 2D segment [p,q] meets the closed (possibly degenerate) triangle t */
static int seg_tri_2d(const double *p, const double *q, const double *t0, const double *t1,
                      const double *t2) {
    if (seg_seg_2d(p, q, t0, t1) || seg_seg_2d(p, q, t1, t2) || seg_seg_2d(p, q, t2, t0))
        return 1;
    /* no boundary contact: the segment is wholly inside or wholly outside */
    if (sd3o_orient2d(t0, t1, t2) != 0) {
        int s0 = sd3o_orient2d(t0, t1, p), s1 = sd3o_orient2d(t1, t2, p),
            s2 = sd3o_orient2d(t2, t0, p);
        if ((s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0)) return 1;
    }
    return 0;
}

/*
 * For coplanar inputs, intersection in 3D is equivalent to intersection in all
 * three coordinate projections: a projection maps shared points to shared
 * points, and at least one projection is injective on the common plane (or
 * line), where a miss in 3D stays a miss.
 */
static int seg_seg_3d(const double *p, const double *q, const double *r, const double *s) {
    if (sd3o_orient3d(p, q, r, s) != 0) return 0;
    for (int k = 0; k < 3; k++) {
        double P[2], Q[2], R[2], S[2];
        proj(p, k, P);
        proj(q, k, Q);
        proj(r, k, R);
        proj(s, k, S);
        if (!seg_seg_2d(P, Q, R, S)) return 0;
    }
    return 1;
}

/* triangle with collinear (or coincident) vertices: all projections degenerate */
static int tri_degenerate(const double *t0, const double *t1, const double *t2) {
    for (int k = 0; k < 3; k++) {
        double A[2], B[2], C[2];
        proj(t0, k, A);
        proj(t1, k, B);
        proj(t2, k, C);
        if (sd3o_orient2d(A, B, C) != 0) return 0;
    }
    return 1;
}

/* closed segment [p,q] meets closed triangle (t0,t1,t2) -- Eq. 4 in sign form */
static int seg_tri_3d(const double *p, const double *q, const double *t0, const double *t1,
                      const double *t2) {
    if (tri_degenerate(t0, t1, t2))
        return seg_seg_3d(p, q, t0, t1) || seg_seg_3d(p, q, t1, t2) || seg_seg_3d(p, q, t2, t0);
    int op = sd3o_orient3d(t0, t1, t2, p), oq = sd3o_orient3d(t0, t1, t2, q);
    if (op * oq > 0) return 0; /* strictly on one side: t outside [0,1] */
    if (op == 0 && oq == 0) {  /* segment in the triangle's plane */
        for (int k = 0; k < 3; k++) {
            double P[2], Q[2], A[2], B[2], C[2];
            proj(p, k, P);
            proj(q, k, Q);
            proj(t0, k, A);
            proj(t1, k, B);
            proj(t2, k, C);
            if (!seg_tri_2d(P, Q, A, B, C)) return 0;
        }
        return 1;
    }
    /* the segment crosses or touches the plane once; the crossing point lies in
     * the closed triangle iff the line pq passes on the same side of (or on)
     * all three directed edges: u, v >= 0 and u + v <= 1 */
    int s0 = sd3o_orient3d(p, q, t0, t1), s1 = sd3o_orient3d(p, q, t1, t2),
        s2 = sd3o_orient3d(p, q, t2, t0);
    return (s0 >= 0 && s1 >= 0 && s2 >= 0) || (s0 <= 0 && s1 <= 0 && s2 <= 0);
}

/* closed triangles A, B (9 doubles each: v0 v1 v2) share a point */
int sd3o_tri_tri_intersect(const double *A, const double *B) {
    /* exact early-out: separated bounding boxes */
    for (int k = 0; k < 3; k++) {
        double alo = fmin(fmin(A[k], A[3 + k]), A[6 + k]), ahi = fmax(fmax(A[k], A[3 + k]), A[6 + k]);
        double blo = fmin(fmin(B[k], B[3 + k]), B[6 + k]), bhi = fmax(fmax(B[k], B[3 + k]), B[6 + k]);
        if (ahi < blo || bhi < alo) return 0;
    }
    for (int i = 0; i < 3; i++)
        if (seg_tri_3d(A + 3 * i, A + 3 * ((i + 1) % 3), B, B + 3, B + 6)) return 1;
    for (int i = 0; i < 3; i++)
        if (seg_tri_3d(B + 3 * i, B + 3 * ((i + 1) % 3), A, A + 3, A + 6)) return 1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Distances (FP64)                                                            */
/* ------------------------------------------------------------------------- */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double *a, const double *b, double *r) {
    r[0] = a[0] - b[0];
    r[1] = a[1] - b[1];
    r[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *r) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* squared distance from point p to closed segment [x0, x1] */
double sd3o_point_seg_d2(const double *p, const double *x0, const double *x1) {
    double v[3], w[3], z[3];
    sub3(x1, x0, v);
    sub3(p, x0, w);
    double c = dot3(v, v);
    double t = c > 0.0 ? clamp01(dot3(w, v) / c) : 0.0;
    for (int i = 0; i < 3; i++) z[i] = w[i] - t * v[i];
    return dot3(z, z);
}

/* squared distance between closed segments [p0,p1] and [q0,q1]:
 * min over the unit square of |r + s u - t v|^2, r = p0 - q0 */
double sd3o_seg_seg_d2(const double *p0, const double *p1, const double *q0, const double *q1) {
    double best = sd3o_point_seg_d2(p0, q0, q1);     /* side s = 0 */
    double x = sd3o_point_seg_d2(p1, q0, q1);        /* side s = 1 */
    if (x < best) best = x;
    x = sd3o_point_seg_d2(q0, p0, p1);               /* side t = 0 */
    if (x < best) best = x;
    x = sd3o_point_seg_d2(q1, p0, p1);               /* side t = 1 */
    if (x < best) best = x;
    double u[3], v[3], r[3];
    sub3(p1, p0, u);
    sub3(q1, q0, v);
    sub3(p0, q0, r);
    double a = dot3(u, u), b = dot3(u, v), c = dot3(v, v), d = dot3(u, r), e = dot3(v, r);
    double D = a * c - b * b;
    if (D > 0.0) { /* interior stationary point */
        double s = (b * e - c * d) / D, t = (a * e - b * d) / D;
        if (s >= 0.0 && s <= 1.0 && t >= 0.0 && t <= 1.0) {
            double w[3];
            for (int i = 0; i < 3; i++) w[i] = r[i] + s * u[i] - t * v[i];
            x = dot3(w, w);
            if (x < best) best = x;
        }
    }
    return best;
}

/* squared distance from p to triangle (x,y,z) when the foot of the
 * perpendicular lies in the closed triangle; +inf otherwise (the boundary is
 * covered by the edge terms) */
double sd3o_vertex_face_d2(const double *p, const double *x, const double *y, const double *z) {
    double e0[3], e1[3], n[3];
    sub3(y, x, e0);
    sub3(z, x, e1);
    cross3(e0, e1, n);
    double nn = dot3(n, n);
    if (nn == 0.0) return INFINITY;
    double w[3], m[3], ek[3], wk[3];
    sub3(p, x, w);
    double h = dot3(n, w);
    /* (e_k x (p - v_k)) . n >= 0 for the three directed edges */
    cross3(e0, w, m);
    if (dot3(m, n) < 0.0) return INFINITY;
    sub3(z, y, ek);
    sub3(p, y, wk);
    cross3(ek, wk, m);
    if (dot3(m, n) < 0.0) return INFINITY;
    sub3(x, z, ek);
    sub3(p, z, wk);
    cross3(ek, wk, m);
    if (dot3(m, n) < 0.0) return INFINITY;
    return h * h / nn;
}

/* squared distance between two closed triangles that do not intersect */
double sd3o_disjoint_pair_d2(const double *A, const double *B) {
    double best = INFINITY, x;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            x = sd3o_seg_seg_d2(A + 3 * i, A + 3 * ((i + 1) % 3), B + 3 * j, B + 3 * ((j + 1) % 3));
            if (x < best) best = x;
        }
    for (int i = 0; i < 3; i++) {
        x = sd3o_vertex_face_d2(A + 3 * i, B, B + 3, B + 6);
        if (x < best) best = x;
        x = sd3o_vertex_face_d2(B + 3 * i, A, A + 3, A + 6);
        if (x < best) best = x;
    }
    return best;
}

/* squared distance between two closed triangles (0 when they intersect) */
double sd3o_pair_d2(const double *A, const double *B) {
    if (sd3o_tri_tri_intersect(A, B)) return 0.0;
    return sd3o_disjoint_pair_d2(A, B);
}

/* ------------------------------------------------------------------------- */
/* Meshes                                                                       */
/* ------------------------------------------------------------------------- */
static void gather(const double *xyz, const int32_t *tri, int64_t t, double *out) {
    for (int k = 0; k < 3; k++) {
        const double *v = xyz + 3 * (int64_t)tri[3 * t + k];
        out[3 * k] = v[0];
        out[3 * k + 1] = v[1];
        out[3 * k + 2] = v[2];
    }
}

/* all pairs: d2 = min over pairs of the pair distance; hit = any pair meets.
 * want: 1 distance (hit is a by-product), 2 intersects only (stops at the
 * first hit).  Returns the number of pair tests run. */
static int64_t mesh_all_pairs(const double *xa, const int32_t *ta, int64_t na, const double *xb,
                              const int32_t *tb, int64_t nb, int want, int threads, double *d2_out,
                              int *hit_out) {
    double best = INFINITY;
    int hit = 0;
    int64_t tests = 0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(threads) reduction(min : best) \
    reduction(| : hit) reduction(+ : tests)
    for (int64_t i = 0; i < na; i++) {
        double A[9], B[9];
        if (want == 2 && __atomic_load_n(hit_out, __ATOMIC_RELAXED)) continue;
        gather(xa, ta, i, A);
        for (int64_t j = 0; j < nb; j++) {
            gather(xb, tb, j, B);
            tests++;
            if (want == 2) {
                if (sd3o_tri_tri_intersect(A, B)) {
                    hit = 1;
                    __atomic_store_n(hit_out, 1, __ATOMIC_RELAXED);
                    break;
                }
            } else {
                int ih = sd3o_tri_tri_intersect(A, B);
                double x = ih ? 0.0 : sd3o_disjoint_pair_d2(A, B);
                if (ih) hit = 1;
                if (x < best) best = x;
            }
        }
    }
    *d2_out = best;
    *hit_out = *hit_out | hit;
    return tests;
}

typedef struct {
    double lo[3], hi[3];
} box;

typedef struct {
    double lb;
    int64_t i, j;
} chunk_pair;

static int cmp_cp(const void *x, const void *y) {
    const chunk_pair *a = x, *b = y;
    if (a->lb < b->lb) return -1;
    if (a->lb > b->lb) return 1;
    if (a->i != b->i) return a->i < b->i ? -1 : 1;
    return (a->j > b->j) - (a->j < b->j);
}

static void chunk_boxes(const double *x, const int32_t *t, int64_t n, int64_t C, box *out) {
    int64_t nc = (n + C - 1) / C;
    for (int64_t c = 0; c < nc; c++) {
        box b;
        for (int k = 0; k < 3; k++) {
            b.lo[k] = INFINITY;
            b.hi[k] = -INFINITY;
        }
        for (int64_t f = c * C; f < n && f < (c + 1) * C; f++)
            for (int v = 0; v < 3; v++)
                for (int k = 0; k < 3; k++) {
                    double q = x[3 * (int64_t)t[3 * f + v] + k];
                    if (q < b.lo[k]) b.lo[k] = q;
                    if (q > b.hi[k]) b.hi[k] = q;
                }
        out[c] = b;
    }
}

/*
 * Exact pruned mode: the same pair routine over a subset of pairs that is
 * guaranteed to contain the minimum.  Triangles are cut into chunks of C
 * consecutive input triangles; the distance between two chunks' bounding
 * boxes is a lower bound of every pair distance inside.  Chunk pairs are
 * visited in increasing bound order and a chunk pair is skipped when its bound
 * exceeds the best pair distance found so far by a margin (1e-9 relative to
 * the distances and box sizes involved) that is far larger than the rounding
 * error of the pair routine, so no skipped pair could have produced a smaller
 * computed value: the result is bit-identical to the all-pairs mode.
 * Intersects visits only chunk pairs whose closed boxes overlap.
 */
static int64_t mesh_pruned(const double *xa, const int32_t *ta, int64_t na, const double *xb,
                           const int32_t *tb, int64_t nb, int want, int threads, double *d2_out,
                           int *hit_out) {
    const int64_t C = 256;
    int64_t nca = (na + C - 1) / C, ncb = (nb + C - 1) / C;
    box *ba = malloc(sizeof(box) * (size_t)nca), *bb = malloc(sizeof(box) * (size_t)ncb);
    chunk_boxes(xa, ta, na, C, ba);
    chunk_boxes(xb, tb, nb, C, bb);
    double ext = 0.0;
    for (int64_t c = 0; c < nca + ncb; c++) {
        box *b = c < nca ? &ba[c] : &bb[c - nca];
        double s = 0.0;
        for (int k = 0; k < 3; k++) s += (b->hi[k] - b->lo[k]) * (b->hi[k] - b->lo[k]);
        if (sqrt(s) > ext) ext = sqrt(s);
    }
    chunk_pair *cp = malloc(sizeof(chunk_pair) * (size_t)(nca * ncb));
    int64_t ncp = 0;
    for (int64_t i = 0; i < nca; i++)
        for (int64_t j = 0; j < ncb; j++) {
            double g2 = 0.0;
            int overlap = 1;
            for (int k = 0; k < 3; k++) {
                double g = 0.0;
                if (bb[j].lo[k] > ba[i].hi[k]) g = bb[j].lo[k] - ba[i].hi[k];
                if (ba[i].lo[k] > bb[j].hi[k]) g = ba[i].lo[k] - bb[j].hi[k];
                if (bb[j].lo[k] > ba[i].hi[k] || ba[i].lo[k] > bb[j].hi[k]) overlap = 0;
                g2 += g * g;
            }
            if (want == 2 && !overlap) continue;
            cp[ncp].lb = sqrt(g2);
            cp[ncp].i = i;
            cp[ncp].j = j;
            ncp++;
        }
    qsort(cp, (size_t)ncp, sizeof(chunk_pair), cmp_cp);
    double best = INFINITY; /* squared */
    int hit = 0;
    int64_t tests = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads) reduction(+ : tests)
    for (int64_t k = 0; k < ncp; k++) {
        double cur;
        int h;
#pragma omp atomic read
        cur = best;
#pragma omp atomic read
        h = hit;
        if (h) continue;
        double bd = sqrt(cur);
        if (want != 2 && cp[k].lb * (1.0 - 1e-9) > bd + 1e-9 * (bd + 2.0 * ext)) continue;
        double A[9], B[9], local = INFINITY;
        int lh = 0;
        for (int64_t f = cp[k].i * C; f < na && f < (cp[k].i + 1) * C && !lh; f++) {
            gather(xa, ta, f, A);
            for (int64_t g = cp[k].j * C; g < nb && g < (cp[k].j + 1) * C; g++) {
                gather(xb, tb, g, B);
                tests++;
                if (want == 2) {
                    if (sd3o_tri_tri_intersect(A, B)) {
                        lh = 1;
                        break;
                    }
                } else {
                    int ih = sd3o_tri_tri_intersect(A, B);
                    double x = ih ? 0.0 : sd3o_disjoint_pair_d2(A, B);
                    if (x < local) local = x;
                    if (ih) lh = 1;
                }
            }
        }
#pragma omp critical(sd3o_best)
        {
            if (local < best) best = local;
            if (lh) hit = 1;
        }
    }
    free(ba);
    free(bb);
    free(cp);
    *d2_out = best;
    *hit_out = hit;
    return tests;
}

/*
 * One geometry pair.  mode 0: all pairs; mode 1: exact pruned.  want 1:
 * distance (+ intersects as a by-product), 2: intersects only.
 * Outputs: *dist (sqrt of the minimum squared pair distance; +inf for an
 * empty mesh; untouched when want == 2), *hit.  Returns pair tests run.
 */
int64_t sd3o_mesh(const double *xa, const int32_t *ta, int64_t na, const double *xb,
                  const int32_t *tb, int64_t nb, int mode, int want, int threads, double *dist,
                  int *hit) {
    double d2 = INFINITY;
    int h = 0;
    int64_t tests = 0;
    if (na > 0 && nb > 0) {
        if (mode == 0)
            tests = mesh_all_pairs(xa, ta, na, xb, tb, nb, want, threads, &d2, &h);
        else
            tests = mesh_pruned(xa, ta, na, xb, tb, nb, want, threads, &d2, &h);
    }
    if (want != 2) *dist = sqrt(d2);
    *hit = h;
    return tests;
}

/* ------------------------------------------------------------------------- */
/* 3D volume (Sec. 3.2.1): the divergence theorem with F = p/3 turns the      */
/* volume integral into a sum over the faces (Eq. 1); on a triangle u v w the */
/* flux of F through the face is u . n / 6 with n = (v - u) x (w - u) (Eq. 2, */
/* counter-clockwise seen from outside), so V = 1/6 sum_i u_i . n_i.          */
/* Evaluated exactly: every coordinate is an integer times 2^e0 (e0 the       */
/* smallest unit in the last place over the mesh), each term is an exact      */
/* integer in units of 2^(3 e0), and the sum is exact.                        */
/* ------------------------------------------------------------------------- */
static void vol_term(const double *xyz, const int32_t *tri, int64_t t, int e0, bn *out) {
    bn U[3], V[3], W[3], a[3], b[3], n[3], p, q;
    for (int k = 0; k < 3; k++) {
        bn_from_double(&U[k], xyz[3 * (int64_t)tri[3 * t] + k], e0);
        bn_from_double(&V[k], xyz[3 * (int64_t)tri[3 * t + 1] + k], e0);
        bn_from_double(&W[k], xyz[3 * (int64_t)tri[3 * t + 2] + k], e0);
    }
    for (int k = 0; k < 3; k++) {
        bn_sub(&a[k], &V[k], &U[k]);
        bn_sub(&b[k], &W[k], &U[k]);
    }
    for (int k = 0; k < 3; k++) {  /* n = a x b */
        int j = (k + 1) % 3, l = (k + 2) % 3;
        bn_mul(&p, &a[j], &b[l]);
        bn_mul(&q, &a[l], &b[j]);
        bn_sub(&n[k], &p, &q);
    }
    memset(out, 0, sizeof *out);
    for (int k = 0; k < 3; k++) {  /* u . n */
        bn_mul(&p, &U[k], &n[k]);
        bn_add(out, out, &p);
    }
}

/*
 * 6 V of one mesh exactly: |6 V| = sum_i limbs[i] 2^(32 i) * 2^(3 e0), with
 * the sign in *neg.  Returns the number of limbs (0 for V = 0) or -1 when an
 * index is out of range.
 */
int sd3o_volume6_exact(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, int threads,
                       uint32_t *limbs, int *neg, int *e0_out) {
    for (int64_t i = 0; i < 3 * nt; i++)
        if (tri[i] < 0 || tri[i] >= nv) return -1;
    int e0 = 1 << 20;
    for (int64_t i = 0; i < 3 * nv; i++)
        if (xyz[i] != 0.0) {
            int e = ulp_exp(xyz[i]);
            if (e < e0) e0 = e;
        }
    if (e0 == (1 << 20)) e0 = 0;
    bn total;
    memset(&total, 0, sizeof total);
    if (threads < 1) threads = 1;
#pragma omp parallel num_threads(threads)
    {
        bn part, term;
        memset(&part, 0, sizeof part);
#pragma omp for schedule(static)
        for (int64_t t = 0; t < nt; t++) {
            vol_term(xyz, tri, t, e0, &term);
            bn_add(&part, &part, &term);
        }
#pragma omp critical
        bn_add(&total, &total, &part);
    }
    for (int i = 0; i < total.n; i++) limbs[i] = total.d[i];
    *neg = total.neg;
    *e0_out = e0;
    return total.n;
}

/* ------------------------------------------------------------------------- */
/* Point in solid: the generalised winding number of a closed, consistently   */
/* oriented mesh around p, the sum of the signed solid angles its triangles   */
/* subtend at p over 4 pi (Van Oosterom and Strackee's formula for the solid  */
/* angle of a triangle).  1 inside, 0 outside, in FP64; meaningful for points */
/* not within rounding distance of the surface.                              */
/* ------------------------------------------------------------------------- */
double sd3o_winding(const double *xyz, const int32_t *tri, int64_t nt, const double *p) {
    double total = 0.0;
    for (int64_t t = 0; t < nt; t++) {
        double a[3], b[3], c[3];
        for (int k = 0; k < 3; k++) {
            a[k] = xyz[3 * (int64_t)tri[3 * t] + k] - p[k];
            b[k] = xyz[3 * (int64_t)tri[3 * t + 1] + k] - p[k];
            c[k] = xyz[3 * (int64_t)tri[3 * t + 2] + k] - p[k];
        }
        double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b)), lc = sqrt(dot3(c, c));
        double bc[3];
        cross3(b, c, bc);
        double num = dot3(a, bc);
        double den = la * lb * lc + dot3(a, b) * lc + dot3(a, c) * lb + dot3(b, c) * la;
        total += 2.0 * atan2(num, den);
    }
    return total / (4.0 * 3.14159265358979323846);
}
