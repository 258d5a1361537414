/*
 * Triangle-mesh part of the oracle (TEST INFRASTRUCTURE ONLY). The paper shows
 * meshes with mirror and shadow effects combined with Gaussians (Sec. 1,
 * Figs. 1 and 3-6) but gives no shading model; the mixed mesh + Gaussian
 * workload uses the definition written out in oracle/mesh.py. This file only
 * holds the brute-force FP64 ray / triangle test (Moller-Trumbore, no
 * back-face culling).
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int tri_hit(const double v0[3], const double v1[3], const double v2[3], const double o[3],
                   const double d[3], double *t_out, double *margin)
{
    double e1[3], e2[3], p[3], s[3], q[3];
    for (int k = 0; k < 3; ++k) { e1[k] = v1[k] - v0[k]; e2[k] = v2[k] - v0[k]; }
    p[0] = d[1] * e2[2] - d[2] * e2[1];
    p[1] = d[2] * e2[0] - d[0] * e2[2];
    p[2] = d[0] * e2[1] - d[1] * e2[0];
    double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    *margin = INFINITY;
    *t_out = -INFINITY;
    if (det == 0.0) return 0;
    double inv = 1.0 / det;
    for (int k = 0; k < 3; ++k) s[k] = o[k] - v0[k];
    double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) * inv;
    q[0] = s[1] * e1[2] - s[2] * e1[1];
    q[1] = s[2] * e1[0] - s[0] * e1[2];
    q[2] = s[0] * e1[1] - s[1] * e1[0];
    double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
    *t_out = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
    /* signed distance (in barycentric units) to the triangle's boundary */
    double m = u < v ? u : v;
    if (1.0 - u - v < m) m = 1.0 - u - v;
    *margin = m;
    return u >= 0.0 && u <= 1.0 && v >= 0.0 && u + v <= 1.0;
}

/* Closest hit with t > t_eps for every ray; t = +inf and tri = -1 on a miss.
 * amb (optional) flags rays that pass within `edge` (barycentric units) of
 * any triangle edge in front of them, where a float32 test may decide
 * differently. */
void orc_mesh_closest(int64_t n_tris, const float *verts, const int32_t *tris, int64_t n_rays,
                      const double *origin, const double *dir, double t_eps, double *t_out, int64_t *tri_out,
                      double edge, int32_t *amb)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < n_rays; ++r) {
        double best = INFINITY;
        int64_t bi = -1;
        int a = 0;
        for (int64_t f = 0; f < n_tris; ++f) {
            double v[3][3];
            for (int c = 0; c < 3; ++c)
                for (int k = 0; k < 3; ++k) v[c][k] = verts[3 * tris[3 * f + c] + k];
            double t, m;
            int h = tri_hit(v[0], v[1], v[2], origin + 3 * r, dir + 3 * r, &t, &m);
            if (t > t_eps && fabs(m) <= edge) a = 1;
            if (h && t > t_eps && t < best) {
                best = t;
                bi = f;
            }
        }
        t_out[r] = best;
        tri_out[r] = bi;
        if (amb) amb[r] = a;
    }
}
