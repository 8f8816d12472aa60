/* Poisson-disk sampling in a rectangle by Bridson's algorithm (SIGGRAPH 2007
 * sketch "Fast Poisson disk sampling in arbitrary dimensions"), seeded by
 * SplitMix64.  Input generation only: no part of the DG method lives here.
 *
 *   int pds_sample(double r, double x0, double y0, double x1, double y1,
 *                  unsigned long long seed, int k,
 *                  const double* fixed, int n_fixed,
 *                  double* out, int cap);
 *
 * Places the n_fixed points first (they seed the active list), then grows the
 * sample from them.  Returns the number of points written to out (x,y pairs),
 * or -1 if cap is too small. */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned long long u64;

static u64 sm_next(u64* s) {
    u64 z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static double sm_unif(u64* s) { return (double)(sm_next(s) >> 11) * (1.0 / 9007199254740992.0); }

int pds_sample(double r, double x0, double y0, double x1, double y1, u64 seed, int k,
               const double* fixed, int n_fixed, double* out, int cap) {
    const double cs = r / sqrt(2.0);
    const long nx = (long)ceil((x1 - x0) / cs), ny = (long)ceil((y1 - y0) / cs);
    int* grid = (int*)malloc(sizeof(int) * nx * ny);
    int* active = (int*)malloc(sizeof(int) * cap);
    int* over = (int*)malloc(sizeof(int) * (n_fixed + 1));
    int n_over = 0, n = 0, n_act = 0;
    u64 st = seed;
    if (!grid || !active || !over) { free(grid); free(active); free(over); return -1; }
    for (long i = 0; i < nx * ny; ++i) grid[i] = -1;

#define CELLX(px) (long)fmin(fmax(floor(((px) - x0) / cs), 0.0), (double)(nx - 1))
#define CELLY(py) (long)fmin(fmax(floor(((py) - y0) / cs), 0.0), (double)(ny - 1))

    for (int f = 0; f < n_fixed; ++f) {
        if (n >= cap) { n = -1; goto done; }
        out[2 * n] = fixed[2 * f];
        out[2 * n + 1] = fixed[2 * f + 1];
        long cx = CELLX(out[2 * n]), cy = CELLY(out[2 * n + 1]);
        if (grid[cy * nx + cx] < 0) grid[cy * nx + cx] = n;
        else over[n_over++] = n;
        active[n_act++] = n;
        ++n;
    }
    if (n_act == 0) {
        out[0] = x0 + (x1 - x0) * sm_unif(&st);
        out[1] = y0 + (y1 - y0) * sm_unif(&st);
        grid[CELLY(out[1]) * nx + CELLX(out[0])] = 0;
        active[n_act++] = 0;
        n = 1;
    }
    while (n_act > 0) {
        int ai = (int)(sm_unif(&st) * n_act);
        if (ai >= n_act) ai = n_act - 1;
        const int p = active[ai];
        const double px = out[2 * p], py = out[2 * p + 1];
        int placed = 0;
        for (int t = 0; t < k && !placed; ++t) {
            const double rad = r * sqrt(1.0 + 3.0 * sm_unif(&st));   /* uniform in annulus area */
            const double ang = 6.283185307179586 * sm_unif(&st);
            const double qx = px + rad * cos(ang), qy = py + rad * sin(ang);
            if (!(qx > x0 && qx < x1 && qy > y0 && qy < y1)) continue;
            const long cx = CELLX(qx), cy = CELLY(qy);
            int ok = grid[cy * nx + cx] < 0;
            for (long dy = -2; dy <= 2 && ok; ++dy)
                for (long dx = -2; dx <= 2 && ok; ++dx) {
                    const long gx = cx + dx, gy = cy + dy;
                    if (gx < 0 || gy < 0 || gx >= nx || gy >= ny) continue;
                    const int q = grid[gy * nx + gx];
                    if (q >= 0) {
                        const double ddx = out[2 * q] - qx, ddy = out[2 * q + 1] - qy;
                        if (ddx * ddx + ddy * ddy < r * r) ok = 0;
                    }
                }
            for (int o = 0; o < n_over && ok; ++o) {
                const double ddx = out[2 * over[o]] - qx, ddy = out[2 * over[o] + 1] - qy;
                if (ddx * ddx + ddy * ddy < r * r) ok = 0;
            }
            if (!ok) continue;
            if (n >= cap) { n = -1; goto done; }
            out[2 * n] = qx;
            out[2 * n + 1] = qy;
            grid[cy * nx + cx] = n;
            active[n_act++] = n;
            ++n;
            placed = 1;
        }
        if (!placed) active[ai] = active[--n_act];
    }
done:
    free(grid);
    free(active);
    free(over);
    return n;
}
