// C-ABI entry points: kernel presets, argument validation, workspace sizing,
// pair enumeration (uniform cell grid) and dispatch of the forward kernels.

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <rocprim/device/device_scan.hpp>

#include "internal.h"
#include "refine.h"
#include "surrogate.h"

namespace sphbi {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

static bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

#define CHECK_HIP(expr)                                                              \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            set_error("%s: %s", #expr, hipGetErrorString(e_));                       \
            return SPHBI_EDEVICE;                                                    \
        }                                                                            \
    } while (0)

// ----------------------------------------------------------------------------
// kernel presets: expand (1 - q/R)^a g(q/R) into monomials of q
// ----------------------------------------------------------------------------
static int expand_piece(int a, const double *g, int ng, double R, double *b) {
    double c[16] = {0};
    c[0] = 1.0;
    int n = 1;
    for (int i = 0; i < a; ++i) {
        for (int j = n; j >= 1; --j) c[j] -= c[j - 1];
        ++n;
    }
    double r[16] = {0};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < ng; ++j) r[i + j] += c[i] * g[j];
    const int deg = n + ng - 2;
    double Rk = 1.0;
    for (int k = 0; k <= deg; ++k) {
        b[k] = r[k] / Rk;
        Rk *= R;
    }
    return deg;
}

static double piece_mass(const double *b, int deg, double R) {   // int_0^R k(q) q dq
    double s = 0.0;
    for (int k = 0; k <= deg; ++k) s += b[k] * pow(R, k + 2) / (k + 2);
    return s;
}

}  // namespace sphbi

using namespace sphbi;

extern "C" {

const char *sphbi_last_error(void) { return g_err; }

void sphbi_default_opts(sphbi_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->precision = SPHBI_FP64;
    o->tau_edge = 1e-4;
}

int sphbi_kernel_preset(int32_t id, sphbi_kernel *out) {
    if (!out) { set_error("sphbi_kernel_preset: out is NULL"); return SPHBI_EINVAL; }
    memset(out, 0, sizeof(*out));
    static const double gC2[2] = {1.0, 4.0};
    static const double gC4[3] = {1.0, 6.0, 35.0 / 3.0};
    static const double gC6[4] = {1.0, 8.0, 25.0, 32.0};
    static const double one[1] = {1.0}, half[1] = {-0.5};
    switch (id) {
    case SPHBI_WENDLAND_C2: out->n_pieces = 1; out->radius[0] = 1.0; out->degree[0] = expand_piece(4, gC2, 2, 1.0, out->b[0]); break;
    case SPHBI_WENDLAND_C4: out->n_pieces = 1; out->radius[0] = 1.0; out->degree[0] = expand_piece(6, gC4, 3, 1.0, out->b[0]); break;
    case SPHBI_WENDLAND_C6: out->n_pieces = 1; out->radius[0] = 1.0; out->degree[0] = expand_piece(8, gC6, 4, 1.0, out->b[0]); break;
    case SPHBI_CUBIC_BSPLINE:
        out->n_pieces = 2;
        out->radius[0] = 1.0;
        out->degree[0] = expand_piece(3, one, 1, 1.0, out->b[0]);
        out->radius[1] = 0.5;
        out->degree[1] = expand_piece(3, half, 1, 0.5, out->b[1]);   // -4 (1/2 - q)^3 = -1/2 (1 - 2q)^3
        break;
    default: set_error("unknown kernel preset %d", id); return SPHBI_EINVAL;
    }
    double mass = 0.0;
    for (int p = 0; p < out->n_pieces; ++p) mass += piece_mass(out->b[p], out->degree[p], out->radius[p]);
    out->c_d = 1.0 / (2.0 * M_PI * mass);
    return SPHBI_OK;
}

}  // extern "C"

namespace sphbi {

static int validate_kernel(const sphbi_kernel *k) {
    if (!k) { set_error("kernel is NULL"); return SPHBI_EINVAL; }
    if (k->n_pieces < 1 || k->n_pieces > 2) { set_error("n_pieces must be 1 or 2"); return SPHBI_EINVAL; }
    for (int p = 0; p < k->n_pieces; ++p) {
        if (k->degree[p] < 0 || k->degree[p] > kMaxDeg) { set_error("degree must be in [0, 11]"); return SPHBI_EINVAL; }
        if (!(k->radius[p] > 0.0 && k->radius[p] <= 1.0)) { set_error("radius must be in (0, 1]"); return SPHBI_EINVAL; }
    }
    if (!isfinite(k->c_d)) { set_error("c_d not finite"); return SPHBI_EINVAL; }
    return SPHBI_OK;
}

KArgs make_kargs(const sphbi_kernel *k, int *deg_out) {
    KArgs K;
    memset(&K, 0, sizeof(K));
    K.npieces = k->n_pieces;
    K.cd = k->c_d;
    int deg = 0;
    for (int p = 0; p < k->n_pieces; ++p) {
        const double R = k->radius[p];
        K.R[p] = R;
        K.iR[p] = 1.0 / R;
        if (k->degree[p] > deg) deg = k->degree[p];
        for (int m = 0; m <= kMaxOrder; ++m) {
            double sv = 0.0, sw = 0.0;
            for (int j = 0; j <= k->degree[p]; ++j) {
                const double b = k->b[p][j];
                K.b[p][j] = b;
                K.bq[p][m][j] = b / (j + 2 + m);
                K.kbq[p][m][j] = j * b / (j + 1 + m);
                sv += b * pow(R, j + 2 + m) / (j + 2 + m);
                sw += j * b * pow(R, j + 1 + m) / (j + 1 + m);
            }
            K.sv[p][m] = sv;
            K.sw[p][m] = sw;
        }
    }
    *deg_out = deg;
    return K;
}

// ----------------------------------------------------------------------------
// pair enumeration kernels
// ----------------------------------------------------------------------------
struct GridDev {
    double x0, y0, icell;
    int nx, ny;
};

__global__ void bbox_partial(int64_t N, const double *__restrict__ px, const double *__restrict__ py,
                             double *__restrict__ part) {
    __shared__ double s[4][256];
    double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        const double x = px[i], y = py[i];
        // fmin and fmax drop NaN: count it as -inf in the minima instead,
        // so that the plan sees a non-finite box
        mnx = fmin(mnx, x == x ? x : -INFINITY); mxx = fmax(mxx, x);
        mny = fmin(mny, y == y ? y : -INFINITY); mxy = fmax(mxy, y);
    }
    s[0][threadIdx.x] = mnx; s[1][threadIdx.x] = mny; s[2][threadIdx.x] = mxx; s[3][threadIdx.x] = mxy;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

__device__ inline void tri_cells(const GridDev &g, const double *__restrict__ tri, int64_t T, int64_t t, double h,
                                 int &cx0, int &cx1, int &cy0, int &cy1) {
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const double x = tri[(2 * v) * T + t], y = tri[(2 * v + 1) * T + t];
        xmin = fmin(xmin, x); xmax = fmax(xmax, x);
        ymin = fmin(ymin, y); ymax = fmax(ymax, y);
    }
    const double fx0 = floor((xmin - h - g.x0) * g.icell), fx1 = floor((xmax + h - g.x0) * g.icell);
    const double fy0 = floor((ymin - h - g.y0) * g.icell), fy1 = floor((ymax + h - g.y0) * g.icell);
    // clamp to the grid; an empty range when the box misses it (also for non-finite input)
    cx0 = (int)fmax(fx0, 0.0);
    cy0 = (int)fmax(fy0, 0.0);
    cx1 = (int)fmin(fx1, (double)(g.nx - 1));
    cy1 = (int)fmin(fy1, (double)(g.ny - 1));
    if (!(fx1 >= 0.0) || !(fy1 >= 0.0) || !(fx0 <= g.nx - 1) || !(fy0 <= g.ny - 1)) { cx1 = cx0 - 1; cy1 = cy0 - 1; }
}

// The plan on the device, so that the host waits once: the particles'
// bounding box from the per-block partials, and from it the grid exactly as
// the host states it in sphbi_grid (cell = h, or extent / 4096 when that is
// larger; nx, ny from the extents).  A non-finite box gives an empty grid
// (the host then reports the coordinates).
struct PlanOut {
    double bb[4];
    double x0, y0, cell;
    int nx, ny;
    unsigned long long total;
};

__global__ __launch_bounds__(256) void plan_grid(int nb, const double *__restrict__ part, double h,
                                                 PlanOut *__restrict__ out) {
    __shared__ double s[4][256];
    double v[4] = {INFINITY, INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nb; b += 256) {
        v[0] = fmin(v[0], part[4 * b]);
        v[1] = fmin(v[1], part[4 * b + 1]);
        v[2] = fmax(v[2], part[4 * b + 2]);
        v[3] = fmax(v[3], part[4 * b + 3]);
    }
    for (int k = 0; k < 4; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double b0 = s[0][0], b1 = s[1][0], b2 = s[2][0], b3 = s[3][0];
        out->bb[0] = b0; out->bb[1] = b1; out->bb[2] = b2; out->bb[3] = b3;
        out->total = 0;
        if (isfinite(b0) && isfinite(b1) && isfinite(b2) && isfinite(b3)) {
            const double ext = fmax(b2 - b0, b3 - b1);
            double cell = h;
            if (ext / cell > 4096.0) cell = ext / 4096.0;
            out->x0 = b0;
            out->y0 = b1;
            out->cell = cell;
            out->nx = (int)floor((b2 - b0) / cell) + 1;
            out->ny = (int)floor((b3 - b1) / cell) + 1;
        } else {
            out->x0 = out->y0 = 0.0;
            out->cell = h;
            out->nx = out->ny = 0;
        }
    }
}

// Grid registrations of the whole mesh (the plan's size query) on the
// device-side grid: one atomic per block of 256 triangles (atomics on one
// address serialise).  A triangle covers at most 4097^2 cells.
__global__ __launch_bounds__(256) void plan_refs(PlanOut *__restrict__ pg, int64_t T, const double *__restrict__ tri,
                                                 double h) {
    __shared__ unsigned long long s_part[4];
    GridDev g;
    g.x0 = pg->x0;
    g.y0 = pg->y0;
    g.icell = 1.0 / pg->cell;
    g.nx = pg->nx;
    g.ny = pg->ny;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long n = 0;
    if (t < T && g.nx > 0 && g.ny > 0) {
        int cx0, cx1, cy0, cy1;
        tri_cells(g, tri, T, t, h, cx0, cx1, cy0, cy1);
        if (cx1 >= cx0 && cy1 >= cy0) n = (unsigned long long)(cx1 - cx0 + 1) * (unsigned long long)(cy1 - cy0 + 1);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) n += __shfl_xor(n, d);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = n;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long b = s_part[0] + s_part[1] + s_part[2] + s_part[3];
        if (b) atomicAdd(&pg->total, b);
    }
}

// Registration of every triangle in the cells its support box covers,
// 16 lanes per triangle (a triangle covers about 30 cells on a mesh of
// triangles a few h across): with one thread per triangle the serial chain
// of atomics was the cost.  FILL = false counts per cell; FILL = true writes
// the triangle into the cell's slot range (in an order the atomics decide;
// cell_sort restores ascending order).
template <bool FILL>
__global__ void tri_ref_cells(GridDev g, int64_t T, const double *__restrict__ tri, double h,
                              int *__restrict__ cursor, const int *__restrict__ cell_start, int *__restrict__ items,
                              int64_t n_refs) {
    const int64_t nthreads = T * 16;
    for (int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < nthreads;
         gid += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = gid >> 4;
        const int sub = (int)(gid & 15);
        int cx0, cx1, cy0, cy1;
        tri_cells(g, tri, T, t, h, cx0, cx1, cy0, cy1);
        if (cx1 < cx0 || cy1 < cy0) continue;
        const int wx = cx1 - cx0 + 1;
        const int64_t n = (int64_t)wx * (cy1 - cy0 + 1);
        for (int64_t k = sub; k < n; k += 16) {
            const int c = (cy0 + (int)(k / wx)) * g.nx + cx0 + (int)(k % wx);
            if (FILL) {
                const int slot = cell_start[c] + atomicAdd(&cursor[c], 1);
                if (slot < n_refs) items[slot] = (int)t;
            } else {
                atomicAdd(&cursor[c], 1);
            }
        }
    }
}

// Every cell's triangles in ascending index order, so that a particle's
// pairs come out sorted (a particle reads the list of its own cell only).
// Here and in the pair kernels a cell list is cut at n_refs, the size of
// the items array: registrations beyond it (a grid planned for other
// triangles or another h) are dropped, never read or written.
//
// A block takes 256 consecutive cells, whose lists are one contiguous range
// of items: staged in LDS when it fits (the usual ~10 entries per cell),
// sorted in place in global memory otherwise.  Shell sort with Ciura's gaps:
// insertion sort for short lists, no quadratic worst case for a cell that
// many large triangles cover.
__device__ inline void shell_sort(int *v, int n) {
    constexpr int gaps[8] = {701, 301, 132, 57, 23, 10, 4, 1};
    for (int gi = 0; gi < 8; ++gi) {
        const int gap = gaps[gi];
        if (gap >= n) continue;
        for (int i = gap; i < n; ++i) {
            const int x = v[i];
            int j = i;
            for (; j >= gap && v[j - gap] > x; j -= gap) v[j] = v[j - gap];
            v[j] = x;
        }
    }
}

constexpr int kSortLds = 8192;       // ints of LDS per block (32 KB)

__global__ __launch_bounds__(256) void cell_sort(int64_t ncell, const int *__restrict__ cell_start,
                                                 int *__restrict__ items, int64_t n_refs) {
    __shared__ int s_items[kSortLds];
    const int64_t c0 = (int64_t)blockIdx.x * 256;
    const int64_t c = c0 + threadIdx.x;
    const int64_t cl = c0 + 256 < ncell ? c0 + 256 : ncell;
    const int a0 = (int)min((int64_t)cell_start[c0], n_refs);
    const int a1 = (int)min((int64_t)cell_start[cl], n_refs);
    const bool staged = a1 - a0 <= kSortLds;           // the same for the whole block
    if (staged) {
        for (int k = threadIdx.x; k < a1 - a0; k += 256) s_items[k] = items[a0 + k];
        __syncthreads();
    }
    if (c < ncell) {
        const int a = cell_start[c];
        const int b = (int)min((int64_t)cell_start[c + 1], n_refs);
        if (b - a >= 2) shell_sort(staged ? s_items + (a - a0) : items + a, b - a);
    }
    if (staged) {
        __syncthreads();
        for (int k = threadIdx.x; k < a1 - a0; k += 256) items[a0 + k] = s_items[k];
    }
}

// Block order for the particle kernels: workgroups go to the eight XCDs in
// turn, so block b runs on XCD b mod 8.  Mapping each XCD's blocks to one
// contiguous range of particles keeps the triangles and cell lists that
// range reads in that XCD's own L2.  A bijection on [0, nb).
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
    const int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Triangle vertices as one 64-byte record each (x0 y0 x1 y1 x2 y2 and two
// pad doubles), so that a candidate test reads one cache line instead of six
// strided doubles.
//
// Also a 32-byte FP32 copy relative to the grid origin (x0 y0 x1 y1 x2 y2,
// a flag, a pad), which decides most candidates with half the loads:
// flag 1 when every coordinate lies within +-m of the origin (m bounds the
// particles' coordinates too) and every edge is at least h long, so that the
// FP32 distance, and the FP32 inside test for a point within h, are within
// the margin the count pass allows for; else 0, and the candidate takes the
// FP64 test.
__global__ void tri_pack(GridDev g, double m, double h, int64_t T, const double *__restrict__ tri,
                         double4 *__restrict__ out, float4 *__restrict__ out32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double v[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = tri[k * T + t];
    out[2 * t] = make_double4(v[0], v[1], v[2], v[3]);
    out[2 * t + 1] = make_double4(v[4], v[5], 0.0, 0.0);
    float r[6];
    bool safe = true;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int f = e == 2 ? 0 : e + 1;
        const double ex = v[2 * f] - v[2 * e], ey = v[2 * f + 1] - v[2 * e + 1];
        safe = safe && ex * ex + ey * ey >= h * h;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double d = v[k] - ((k & 1) ? g.y0 : g.x0);
        safe = safe && fabs(d) <= m;          // false for NaN and infinities too
        r[k] = safe ? (float)d : 0.0f;
    }
    out32[2 * t] = make_float4(r[0], r[1], r[2], r[3]);
    out32[2 * t + 1] = make_float4(r[4], r[5], safe ? 1.0f : 0.0f, 0.0f);
}

// Whether (x, y) is within sqrt(h2) of triangle t: the squared distance
// (0 inside) compared with h2.  (A bounding-box rejection first, which
// removes a third of the candidates on a covering mesh, measured no faster:
// the kernel is bound by the candidates' 64-byte loads, not the tests.)
__device__ inline bool near_tri(double x, double y, const double4 *__restrict__ tv, int t, double h2) {
    const double4 va = tv[2 * t], vb = tv[2 * t + 1];
    const double x0 = va.x, y0 = va.y, x1 = va.z, y1 = va.w, x2 = vb.x, y2 = vb.y;
    const double c0 = (x1 - x0) * (y - y0) - (y1 - y0) * (x - x0);
    const double c1 = (x2 - x1) * (y - y1) - (y2 - y1) * (x - x1);
    const double c2 = (x0 - x2) * (y - y2) - (y0 - y2) * (x - x2);
    if ((c0 >= 0.0 && c1 >= 0.0 && c2 >= 0.0) || (c0 <= 0.0 && c1 <= 0.0 && c2 <= 0.0)) return true;
    double best = INFINITY;
    const double ex[3] = {x0, x1, x2}, ey[3] = {y0, y1, y2};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double ax = ex[e], ay = ey[e], ux = ex[(e + 1) % 3], uy = ey[(e + 1) % 3];
        const double dx = ux - ax, dy = uy - ay;
        const double L = dx * dx + dy * dy;
        double s = L > 0.0 ? ((x - ax) * dx + (y - ay) * dy) / L : 0.0;
        s = fmin(fmax(s, 0.0), 1.0);
        const double qx = ax + s * dx - x, qy = ay + s * dy - y;
        best = fmin(best, qx * qx + qy * qy);
    }
    return best < h2;
}

__device__ inline int particle_cell(const GridDev &g, double x, double y) {
    int cx = (int)fmin(fmax(floor((x - g.x0) * g.icell), 0.0), (double)(g.nx - 1));
    int cy = (int)fmin(fmax(floor((y - g.y0) * g.icell), 0.0), (double)(g.ny - 1));
    return cy * g.nx + cx;
}

// Pairs per particle.  A particle whose cell lists at most 64 triangles also
// keeps the bit mask of those that pass, so that pair_fill need not test them
// again.
// The squared distance from (x, y) to a triangle in FP32 (0 inside), the
// same steps as near_tri with the reciprocal estimate for the quotient.
__device__ inline float dist2_tri32(float x, float y, const float4 *__restrict__ tv32, int t, bool &safe) {
    const float4 va = tv32[2 * t], vb = tv32[2 * t + 1];
    safe = vb.z != 0.0f;
    const float x0 = va.x, y0 = va.y, x1 = va.z, y1 = va.w, x2 = vb.x, y2 = vb.y;
    const float c0 = (x1 - x0) * (y - y0) - (y1 - y0) * (x - x0);
    const float c1 = (x2 - x1) * (y - y1) - (y2 - y1) * (x - x1);
    const float c2 = (x0 - x2) * (y - y2) - (y0 - y2) * (x - x2);
    if ((c0 >= 0.0f && c1 >= 0.0f && c2 >= 0.0f) || (c0 <= 0.0f && c1 <= 0.0f && c2 <= 0.0f)) return 0.0f;
    float best = INFINITY;
    const float ex[3] = {x0, x1, x2}, ey[3] = {y0, y1, y2};
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const float ax = ex[e], ay = ey[e], ux = ex[(e + 1) % 3], uy = ey[(e + 1) % 3];
        const float dx = ux - ax, dy = uy - ay;
        const float L = dx * dx + dy * dy;
        float sp = L > 0.0f ? ((x - ax) * dx + (y - ay) * dy) * __builtin_amdgcn_rcpf(L) : 0.0f;
        sp = fminf(fmaxf(sp, 0.0f), 1.0f);
        const float qx = ax + sp * dx - x, qy = ay + sp * dy - y;
        best = fminf(best, qx * qx + qy * qy);
    }
    return best;
}

// Pairs per particle.  A candidate is decided by its FP32 distance when that
// is below lo2 or above hi2 (the support radius less or plus the FP32 error
// bound, squared); the FP64 test decides the others and the triangles far
// from the grid.  A particle whose cell lists at most 64 triangles also keeps
// the bit mask of those that pass, so that pair_fill need not test them again.
//
// outside (nullable): set when a particle lies outside the grid's cells (or
// has a non-finite coordinate); its cell is then clamped to the border and
// pairs with triangles registered only beyond the grid are missed, so a
// list counted on a grid planned for other positions must be planned again.
__global__ void pair_count(GridDev g, int64_t N, const double *__restrict__ px, const double *__restrict__ py,
                           const double4 *__restrict__ tv, const float4 *__restrict__ tv32, double h2, float lo2,
                           float hi2, const int *__restrict__ cell_start, const int *__restrict__ items,
                           int64_t n_refs, int64_t *__restrict__ counts, uint64_t *__restrict__ mask,
                           int *__restrict__ outside) {
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double x = px[i], y = py[i];
    if (outside) {
        const double fx = floor((x - g.x0) * g.icell), fy = floor((y - g.y0) * g.icell);
        if (!(fx >= 0.0 && fx <= g.nx - 1 && fy >= 0.0 && fy <= g.ny - 1)) *outside = 1;
    }
    const float xr = (float)(x - g.x0), yr = (float)(y - g.y0);
    const int c = particle_cell(g, x, y);
    const int k0 = cell_start[c], k1 = (int)min((int64_t)cell_start[c + 1], n_refs);
    int64_t n = 0;
    uint64_t m = 0;
    for (int k = k0; k < k1; ++k) {
        const int t = items[k];
        bool safe;
        const float d2 = dist2_tri32(xr, yr, tv32, t, safe);
        const bool pass = safe && d2 < lo2 ? true : (safe && d2 > hi2 ? false : near_tri(x, y, tv, t, h2));
        if (pass) {
            ++n;
            m |= (uint64_t)1 << ((k - k0) & 63);
        }
    }
    counts[i] = n;
    mask[i] = m;
}

// The cell lists are sorted, so every particle's pairs come out in ascending
// triangle order.
__global__ void pair_fill(GridDev g, int64_t N, const double *__restrict__ px, const double *__restrict__ py,
                          const double4 *__restrict__ tv, double h2, const int *__restrict__ cell_start,
                          const int *__restrict__ items, int64_t n_refs, const uint64_t *__restrict__ mask,
                          const int64_t *__restrict__ offsets, int32_t *__restrict__ tri_idx, int64_t cap) {
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double x = px[i], y = py[i];
    const int c = particle_cell(g, x, y);
    const int64_t q1 = offsets[i + 1] < cap ? offsets[i + 1] : cap;
    const int k0 = cell_start[c], k1 = (int)min((int64_t)cell_start[c + 1], n_refs);
    int64_t q = offsets[i] > 0 ? offsets[i] : 0;
    if (k1 - k0 <= 64) {
        for (uint64_t m = mask[i]; m && q < q1; m &= m - 1) tri_idx[q++] = items[k0 + __builtin_ctzll(m)];
    } else {
        for (int k = k0; k < k1 && q < q1; ++k) {
            const int t = items[k];
            if (near_tri(x, y, tv, t, h2)) tri_idx[q++] = t;
        }
    }
}

struct WsLayout {
    size_t cell_start, cursor, items, tri4, tri32, mask, flag, scan_tmp, scan_tmp_bytes, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int layout(const sphbi_grid *g, int64_t N, int64_t T, WsLayout *L) {
    const size_t ncell = (size_t)g->nx * g->ny;
    size_t t1 = 0, t2 = 0;
    (void)rocprim::exclusive_scan(nullptr, t1, (int *)nullptr, (int *)nullptr, 0, (size_t)(ncell + 1),
                                  rocprim::plus<int>());
    (void)rocprim::inclusive_scan(nullptr, t2, (int64_t *)nullptr, (int64_t *)nullptr, (size_t)(N > 0 ? N : 1),
                                  rocprim::plus<int64_t>());
    size_t o = 0;
    L->cell_start = o; o = align256(o + (ncell + 1) * sizeof(int));
    L->cursor = o; o = align256(o + (ncell + 1) * sizeof(int));
    L->items = o; o = align256(o + (size_t)(g->n_refs > 0 ? g->n_refs : 1) * sizeof(int));
    L->tri4 = o; o = align256(o + (size_t)(T > 0 ? T : 1) * 8 * sizeof(double));
    L->tri32 = o; o = align256(o + (size_t)(T > 0 ? T : 1) * 8 * sizeof(float));
    L->mask = o; o = align256(o + (size_t)(N > 0 ? N : 1) * sizeof(uint64_t));
    L->flag = o; o = align256(o + sizeof(int));
    L->scan_tmp = o;
    L->scan_tmp_bytes = t1 > t2 ? t1 : t2;
    o = align256(o + L->scan_tmp_bytes);
    L->total = o;
    return SPHBI_OK;
}

static int check_pairlist_args(int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                               double h) {
    if (N < 0 || T < 0) { set_error("negative size"); return SPHBI_EINVAL; }
    if (!(h > 0.0) || !isfinite(h)) { set_error("h must be positive and finite"); return SPHBI_EINVAL; }
    if (N > 0 && (!px || !py)) { set_error("particle arrays are NULL"); return SPHBI_EINVAL; }
    if (T > 0 && !tri) { set_error("triangle array is NULL"); return SPHBI_EINVAL; }
    if (!aligned8(px) || !aligned8(py) || !aligned8(tri)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (N > kMaxItems || T > kMaxItems) {
        set_error("more than %lld particles or triangles in one call", (long long)kMaxItems);
        return SPHBI_EUNSUPPORTED;
    }
    return SPHBI_OK;
}

static GridDev to_dev(const sphbi_grid *g) {
    GridDev d;
    d.x0 = g->x0; d.y0 = g->y0; d.icell = 1.0 / g->cell; d.nx = g->nx; d.ny = g->ny;
    return d;
}

}  // namespace sphbi

extern "C" {

int sphbi_pairlist_plan(int64_t N, const double *px, const double *py, int64_t T, const double *tri, double h,
                        sphbi_grid *grid, size_t *ws_bytes, void *stream) {
    int rc = check_pairlist_args(N, px, py, T, tri, h);
    if (rc) return rc;
    if (!grid || !ws_bytes) { set_error("grid/ws_bytes outputs are NULL"); return SPHBI_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    memset(grid, 0, sizeof(*grid));
    void *tmp = nullptr;
    if (N > 0) {
        const int nb = (int)((N + 255) / 256 < 1024 ? (N + 255) / 256 : 1024);
        CHECK_HIP(hipMallocAsync(&tmp, sizeof(double) * 4 * nb + sizeof(PlanOut), s));
        PlanOut *po = (PlanOut *)((char *)tmp + sizeof(double) * 4 * nb);
        hipLaunchKernelGGL(bbox_partial, dim3(nb), dim3(256), 0, s, N, px, py, (double *)tmp);
        hipLaunchKernelGGL(plan_grid, dim3(1), dim3(256), 0, s, nb, (const double *)tmp, h, po);
        if (T > 0) hipLaunchKernelGGL(plan_refs, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, po, T, tri, h);
        CHECK_HIP(hipGetLastError());
        PlanOut ho;
        CHECK_HIP(hipMemcpyAsync(&ho, po, sizeof(ho), hipMemcpyDeviceToHost, s));
        CHECK_HIP(hipStreamSynchronize(s));
        if (!isfinite(ho.bb[0]) || !isfinite(ho.bb[1]) || !isfinite(ho.bb[2]) || !isfinite(ho.bb[3])) {
            (void)hipFreeAsync(tmp, s);
            set_error("non-finite particle coordinates");
            return SPHBI_EINVAL;
        }
        if (ho.total > (unsigned long long)INT32_MAX) {
            (void)hipFreeAsync(tmp, s);
            set_error("grid registrations exceed 2^31");
            return SPHBI_EUNSUPPORTED;
        }
        grid->x0 = ho.x0;
        grid->y0 = ho.y0;
        grid->cell = ho.cell;
        grid->nx = ho.nx;
        grid->ny = ho.ny;
        grid->n_refs = (int64_t)ho.total;
    } else {
        // no particles: the one-cell grid at the origin
        grid->cell = h;
        grid->nx = grid->ny = 1;
    }
    if (tmp) CHECK_HIP(hipFreeAsync(tmp, s));
    WsLayout L;
    layout(grid, N, T, &L);
    *ws_bytes = L.total;
    return SPHBI_OK;
}

}  // extern "C"

namespace sphbi {

// count, and with build_cells the grid's cell lists before it (recount
// reuses those a count call left in ws)
static int pairlist_count_impl(int64_t N, const double *px, const double *py, int64_t T, const double *tri, double h,
                               const sphbi_grid *grid, void *ws, size_t ws_bytes, int64_t *offsets, int64_t *n_pairs,
                               void *stream, bool build_cells) {
    int rc = check_pairlist_args(N, px, py, T, tri, h);
    if (rc) return rc;
    if (!grid || !n_pairs || !offsets) { set_error("grid/offsets/n_pairs is NULL"); return SPHBI_EINVAL; }
    if (grid->nx <= 0 || grid->ny <= 0 || !(grid->cell > 0)) { set_error("grid not planned"); return SPHBI_EINVAL; }
    WsLayout L;
    layout(grid, N, T, &L);
    if (!ws || ws_bytes < L.total) { set_error("workspace too small (%zu < %zu)", ws_bytes, L.total); return SPHBI_ENOWORKSPACE; }
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int *cell_start = (int *)(w + L.cell_start), *cursor = (int *)(w + L.cursor), *items = (int *)(w + L.items);
    double4 *tri4 = (double4 *)(w + L.tri4);
    // FP32 pre-test: coordinates relative to the grid origin within +-m_fp32
    // (twice the grid's extent), each rounded with error <= m 2^-24 =: eta/2.
    // The foot point of a segment is then off by at most about 12 eta/2 per
    // component (the differences, the projection with its 1-ulp reciprocal,
    // the product and the sums; an error in the projection parameter moves
    // the foot along the segment, which changes the distance only to second
    // order), and for a point within h of a triangle whose edges are all at
    // least h long the FP32 inside test errs only for points within 6 eta of
    // an edge line.  So the FP32 distance is within e = 32 m 2^-24 + 4 h 2^-24
    // of the exact one (a generous bound).  Below (h - e)^2 a candidate
    // passes, above (h + e)^2 it fails, in between the FP64 test decides; the
    // squares are rounded outwards.  Beyond m = 2^20 h the second-order term
    // is no longer small and every candidate takes the FP64 test.
    const double m_fp32 = 2.0 * (double)(grid->nx > grid->ny ? grid->nx : grid->ny) * grid->cell + 2.0 * h;
    const double e_fp32 = (32.0 * m_fp32 + 4.0 * h) * 0x1p-24;
    const double lo = h - e_fp32 > 0.0 ? h - e_fp32 : 0.0;
    float lo2 = nextafterf((float)(lo * lo * (1.0 - 0x1p-20)), 0.0f);
    float hi2 = nextafterf((float)((h + e_fp32) * (h + e_fp32) * (1.0 + 0x1p-20)), INFINITY);
    if (!(m_fp32 <= 0x1p20 * h)) {
        lo2 = 0.0f;
        hi2 = INFINITY;
    }
    const size_t ncell = (size_t)grid->nx * grid->ny;
    GridDev g = to_dev(grid);
    // 16 lanes per triangle, grid-stride beyond 2^16 blocks
    const int64_t rb = (T * 16 + 255) / 256;
    const unsigned ref_blocks = (unsigned)(rb < 65536 ? (rb > 0 ? rb : 1) : 65536);
    if (build_cells) {
        CHECK_HIP(hipMemsetAsync(cursor, 0, (ncell + 1) * sizeof(int), s));
        if (T > 0) {
            hipLaunchKernelGGL(tri_pack, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, g, m_fp32, h, T, tri,
                               tri4, (float4 *)(w + L.tri32));
            hipLaunchKernelGGL(tri_ref_cells<false>, dim3(ref_blocks), dim3(256), 0, s, g, T, tri, h, cursor,
                               (const int *)nullptr, (int *)nullptr, (int64_t)0);
        }
        CHECK_HIP(hipGetLastError());
        size_t tb = L.scan_tmp_bytes;
        CHECK_HIP(rocprim::exclusive_scan(w + L.scan_tmp, tb, cursor, cell_start, 0, (size_t)(ncell + 1),
                                          rocprim::plus<int>(), s));
        CHECK_HIP(hipMemsetAsync(cursor, 0, (ncell + 1) * sizeof(int), s));
        if (T > 0) {
            hipLaunchKernelGGL(tri_ref_cells<true>, dim3(ref_blocks), dim3(256), 0, s, g, T, tri, h, cursor,
                               cell_start, items, grid->n_refs);
            hipLaunchKernelGGL(cell_sort, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, (int64_t)ncell,
                               cell_start, items, grid->n_refs);
        }
        CHECK_HIP(hipGetLastError());
    }
    // recount: a particle outside the grid's cells may have pairs the cell
    // lists do not hold
    int *outside = build_cells ? nullptr : (int *)(w + L.flag);
    if (outside) CHECK_HIP(hipMemsetAsync(outside, 0, sizeof(int), s));
    CHECK_HIP(hipMemsetAsync(offsets, 0, sizeof(int64_t), s));
    if (N > 0) {
        hipLaunchKernelGGL(pair_count, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, g, N, px, py,
                           (const double4 *)tri4, (const float4 *)(w + L.tri32), h * h, lo2, hi2, cell_start, items,
                           grid->n_refs, offsets + 1,
                           (uint64_t *)(w + L.mask), outside);
        CHECK_HIP(hipGetLastError());
        size_t tb = L.scan_tmp_bytes;
        CHECK_HIP(rocprim::inclusive_scan(w + L.scan_tmp, tb, offsets + 1, offsets + 1, (size_t)N,
                                          rocprim::plus<int64_t>(), s));
    }
    int out_h = 0;
    CHECK_HIP(hipMemcpyAsync(n_pairs, offsets + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (outside) CHECK_HIP(hipMemcpyAsync(&out_h, outside, sizeof(int), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (out_h) {
        set_error("particles outside the planned grid (or not finite): plan again");
        return SPHBI_EGRID;
    }
    return SPHBI_OK;
}

}  // namespace sphbi

extern "C" {

int sphbi_pairlist_count(int64_t N, const double *px, const double *py, int64_t T, const double *tri, double h,
                         const sphbi_grid *grid, void *ws, size_t ws_bytes, int64_t *offsets, int64_t *n_pairs,
                         void *stream) {
    return pairlist_count_impl(N, px, py, T, tri, h, grid, ws, ws_bytes, offsets, n_pairs, stream, true);
}

int sphbi_pairlist_recount(int64_t N, const double *px, const double *py, int64_t T, const double *tri, double h,
                           const sphbi_grid *grid, void *ws, size_t ws_bytes, int64_t *offsets, int64_t *n_pairs,
                           void *stream) {
    return pairlist_count_impl(N, px, py, T, tri, h, grid, ws, ws_bytes, offsets, n_pairs, stream, false);
}

int sphbi_pairlist_fill(int64_t N, const double *px, const double *py, int64_t T, const double *tri, double h,
                        const sphbi_grid *grid, void *ws, size_t ws_bytes, const int64_t *offsets, int32_t *tri_idx,
                        int64_t cap, void *stream) {
    int rc = check_pairlist_args(N, px, py, T, tri, h);
    if (rc) return rc;
    if (!grid || !offsets || (cap > 0 && !tri_idx)) { set_error("grid/offsets/tri_idx is NULL"); return SPHBI_EINVAL; }
    WsLayout L;
    layout(grid, N, T, &L);
    if (!ws || ws_bytes < L.total) { set_error("workspace too small"); return SPHBI_ENOWORKSPACE; }
    hipStream_t s = (hipStream_t)stream;
    int64_t total = 0;
    CHECK_HIP(hipMemcpyAsync(&total, offsets + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    CHECK_HIP(hipStreamSynchronize(s));
    if (total > cap) { set_error("tri_idx capacity %lld < %lld pairs", (long long)cap, (long long)total); return SPHBI_ECAPACITY; }
    char *w = (char *)ws;
    GridDev g = to_dev(grid);
    if (N > 0)
        hipLaunchKernelGGL(pair_fill, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, g, N, px, py,
                           (const double4 *)(w + L.tri4), h * h, (const int *)(w + L.cell_start),
                           (const int *)(w + L.items), grid->n_refs, (const uint64_t *)(w + L.mask), offsets,
                           tri_idx, cap);
    CHECK_HIP(hipGetLastError());
    return SPHBI_OK;
}

size_t sphbi_integrate_workspace(int64_t T) { return records_bytes(T) + 256 + dd_records_bytes(T); }

static int check_common(const sphbi_kernel *kernel, const sphbi_opts *opts, sphbi_opts *o, double h, int32_t n_nodes,
                        int64_t N, int64_t T, int64_t n_pairs) {
    int rc = validate_kernel(kernel);
    if (rc) return rc;
    sphbi_default_opts(o);
    if (opts) *o = *opts;
    if (o->precision != SPHBI_FP64 && o->precision != SPHBI_MIXED) { set_error("unknown precision %d", o->precision); return SPHBI_EINVAL; }
    if (o->refine != SPHBI_REFINE_AUTO && o->refine != SPHBI_REFINE_OFF && o->refine != SPHBI_REFINE_ALL) {
        set_error("unknown refine mode %d", o->refine);
        return SPHBI_EINVAL;
    }
    if (!(o->refine_gate >= 0.0)) { set_error("refine_gate must be >= 0 (0 = default)"); return SPHBI_EINVAL; }
    if (!(o->tau_edge >= 0.0) || !isfinite(o->tau_edge)) { set_error("tau_edge must be finite and >= 0"); return SPHBI_EINVAL; }
    if (!(h > 0.0) || !isfinite(h)) { set_error("h must be positive and finite"); return SPHBI_EINVAL; }
    if (n_nodes != 1 && n_nodes != 3 && n_nodes != 10) { set_error("n_nodes must be 1, 3 or 10"); return SPHBI_EINVAL; }
    if (N < 0 || T < 0 || n_pairs < 0) { set_error("negative size"); return SPHBI_EINVAL; }
    if (N > kMaxItems || T > kMaxItems) {
        set_error("more than %lld particles or triangles in one call", (long long)kMaxItems);
        return SPHBI_EUNSUPPORTED;
    }
    return SPHBI_OK;
}

}  // extern "C"

namespace sphbi {

// sphbi_field_prepare, and zeroing of the refinement counter (nullable)
static int field_prepare(double h, int32_t n_nodes, int64_t T, const double *tri, const double *nodal, double *rec,
                         size_t rec_bytes, void *stream, unsigned long long *count) {
    if (!(h > 0.0) || !isfinite(h)) { set_error("h must be positive and finite"); return SPHBI_EINVAL; }
    if (n_nodes != 1 && n_nodes != 3 && n_nodes != 10) { set_error("n_nodes must be 1, 3 or 10"); return SPHBI_EINVAL; }
    if (T < 0) { set_error("negative size"); return SPHBI_EINVAL; }
    if (T > kMaxItems) { set_error("more than %lld triangles in one call", (long long)kMaxItems); return SPHBI_EUNSUPPORTED; }
    if (T == 0) return SPHBI_OK;
    if (!tri || !nodal || !rec) { set_error("triangle/nodal/record arrays are NULL"); return SPHBI_EINVAL; }
    if (!aligned8(tri) || !aligned8(nodal) || !aligned8(rec)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (rec_bytes < records_bytes(T) + 256) {               // the records and the refinement counter
        set_error("record buffer too small (%zu < %zu)", rec_bytes, records_bytes(T) + 256);
        return SPHBI_ENOWORKSPACE;
    }
    const int order = n_nodes == 1 ? 0 : (n_nodes == 3 ? 1 : 3);
    return launch_prepare(order, T, tri, nodal, h, rec, (hipStream_t)stream, count);
}

}  // namespace sphbi

extern "C" {

int sphbi_field_prepare(double h, int32_t n_nodes, int64_t T, const double *tri, const double *nodal, double *rec,
                        size_t rec_bytes, void *stream) {
    return field_prepare(h, n_nodes, T, tri, nodal, rec, rec_bytes, stream, nullptr);
}

int sphbi_integrate_prepared(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, int32_t n_nodes,
                             int64_t N, const double *px, const double *py, int64_t T, const double *rec,
                             const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, double *I, double *Gx,
                             double *Gy, double *per_pair, void *stream) {
    sphbi_opts o;
    int rc = check_common(kernel, opts, &o, h, n_nodes, N, T, n_pairs);
    if (rc) return rc;
    if (N > 0 && (!px || !py || !offsets || !I || !Gx || !Gy)) { set_error("particle arrays are NULL"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && (!tri_idx || !rec)) { set_error("pair/record arrays are NULL"); return SPHBI_EINVAL; }
    const void *ptrs[] = {px, py, rec, offsets, tri_idx, I, Gx, Gy, per_pair};
    for (const void *p : ptrs)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (N == 0) return SPHBI_OK;
    int deg = 0;
    const KArgs K = make_kargs(kernel, &deg);
    const int order = n_nodes == 1 ? 0 : (n_nodes == 3 ? 1 : 3);
    return launch_forward(order, deg, o.precision, o.tau_edge, K, refine_off(), h, N, px, py, offsets, tri_idx,
                          n_pairs, T, rec, I, Gx, Gy, per_pair, (hipStream_t)stream, o.pair_status);
}

}  // extern "C"

namespace sphbi {

// Default thresholds of the conditioning gate on Kf kappa^order (see
// sphbi_opts), G = G0 (141 / Kf)^a, 141 being Kf of Wendland C2.  Fitted to
// the errors measured against the double-double path, per pair and per
// particle, on covering meshes (512^2 particles, aspect ratio 20 and 60,
// cubic and linear fields, three seeds) and on 0.5-degree slivers with
// particles 1e-8..1e-2 h from edges and vertices:
//  * FP64, cubic fields: G0 = 3e6, a = 1.65.  Wendland C2 keeps the headline
//    mesh of 2^20 particles unrefined (largest Kf kappa^3 2.2e6, error
//    4.8e-13); Wendland C4 needs G <= 1e5 to stay within 1e-12 per particle
//    (with 2.3e5 the sums of ~5.5 pairs each within 8.5e-13 reached
//    1.0-1.3e-12); C6 and the slivers are refined almost wholly either way.
//  * FP64, linear fields (they lose kappa^1, not kappa^3): G0 = 3e8, the same
//    a; every preset kernel stays within 1e-12 (largest kept error 6.2e-13,
//    Wendland C6 on a covering mesh, where the cubic fields' threshold sent
//    two thirds of the pairs to double-double) while the C6 slivers are
//    still all refined.
//  * Mixed: G0 = 1e9, a = 1.25, which holds the 1e-6 target.
constexpr double kGateFP64 = 3e6, kGateFP64Linear = 3e8, kGateMixed = 1e9;
constexpr double kGateExpFP64 = 1.65, kGateExpMixed = 1.25;

// Kf = sum_p sum_k |b_pk| R_p^(k+2)/(k+2) / |sum_p sum_k b_pk R_p^(k+2)/(k+2)|:
// the cancellation of the kernel's monomial form in the integral over the
// support disc.
static double kernel_cancellation(const KArgs &K) {
    double sa = 0.0, s = 0.0;
    for (int p = 0; p < K.npieces; ++p)
        for (int k = 0; k <= kMaxDeg; ++k) {
            const double t = K.b[p][k] * pow(K.R[p], k + 2) / (k + 2);
            sa += fabs(t);
            s += t;
        }
    return s != 0.0 ? sa / fabs(s) : INFINITY;
}

RefineGate make_gate(const sphbi_opts &o, int order, const KArgs &K) {
    if (o.refine != SPHBI_REFINE_AUTO || order == 0) return refine_off();
    const double kf = kernel_cancellation(K);
    const bool mixed = o.precision == SPHBI_MIXED;
    const double g0 = mixed ? kGateMixed : (order == 1 ? kGateFP64Linear : kGateFP64);
    const double thr = o.refine_gate > 0.0 ? o.refine_gate
                                           : g0 * pow(141.0 / kf, mixed ? kGateExpMixed : kGateExpFP64);
    if (!isfinite(thr)) return refine_off();
    const double g = thr / kf;
    return RefineGate{order, 0, g * g};
}

int integrate_run(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, int32_t n_nodes, int64_t N,
                  const double *px, const double *py, int64_t T, const double *tri, const double *nodal, double *rec,
                  size_t rec_bytes, const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, double *I,
                  double *Gx, double *Gy, double *per_pair, void *stream) {
    sphbi_opts o;
    sphbi_default_opts(&o);
    if (opts) o = *opts;
    int deg = 0;
    const KArgs K = make_kargs(kernel, &deg);
    const int order = n_nodes == 1 ? 0 : (n_nodes == 3 ? 1 : 3);
    hipStream_t s = (hipStream_t)stream;
    // the double-double records of the refinement pass, behind the records
    // and the counter when the storage holds them (else built per pair)
    double *rec_dd = rec_bytes >= records_bytes(T) + 256 + dd_records_bytes(T)
                         ? (double *)((char *)rec + records_bytes(T) + 256)
                         : nullptr;
    // the refinement counter and the refinement pass's window counter sit
    // behind the records (storage that holds them: T = 0 may come without)
    unsigned long long *count = rec && rec_bytes >= records_bytes(T) + 256
                                    ? (unsigned long long *)((char *)rec + records_bytes(T))
                                    : nullptr;
    if (o.refine == SPHBI_REFINE_ALL)
        return launch_refine(order, deg, K, refine_off(), true, h, N, px, py, offsets, tri_idx, n_pairs, T, tri, nodal, I,
                             Gx, Gy, per_pair, s, o.pair_status, rec_dd, count ? count + 1 : nullptr);
    RefineGate gate = T > 0 ? make_gate(o, order, K) : refine_off();
    gate.count = count;
    int rc = field_prepare(h, n_nodes, T, tri, nodal, rec, rec_bytes, stream, gate.order ? count : nullptr);
    if (rc) return rc;
    rc = launch_forward(order, deg, o.precision, o.tau_edge, K, gate, h, N, px, py, offsets, tri_idx, n_pairs, T, rec,
                        I, Gx, Gy, per_pair, s, o.pair_status);
    if (rc || !gate.order) return rc;
    return launch_refine(order, deg, K, gate, false, h, N, px, py, offsets, tri_idx, n_pairs, T, tri, nodal, I, Gx, Gy,
                         per_pair, s, o.pair_status, rec_dd, count + 1);
}

int check_integrate_args(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, int32_t n_nodes, int64_t N,
                         const double *px, const double *py, int64_t T, const double *tri, const double *nodal,
                         const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, const double *I,
                         const double *Gx, const double *Gy, const double *per_pair) {
    sphbi_opts o;
    int rc = check_common(kernel, opts, &o, h, n_nodes, N, T, n_pairs);
    if (rc) return rc;
    if (N > 0 && (!px || !py || !offsets || !I || !Gx || !Gy)) { set_error("particle arrays are NULL"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && (!tri_idx || !tri || !nodal)) { set_error("pair/triangle arrays are NULL"); return SPHBI_EINVAL; }
    const void *ptrs[] = {px, py, tri, nodal, offsets, tri_idx, I, Gx, Gy, per_pair};
    for (const void *p : ptrs)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    return SPHBI_OK;
}

}  // namespace sphbi

extern "C" {

int sphbi_integrate(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, int32_t n_nodes, int64_t N,
                    const double *px, const double *py, int64_t T, const double *tri, const double *nodal,
                    const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, double *I, double *Gx,
                    double *Gy, double *per_pair, void *ws, size_t ws_bytes, void *stream) {
    int rc = check_integrate_args(kernel, opts, h, n_nodes, N, px, py, T, tri, nodal, offsets, tri_idx, n_pairs, I,
                                  Gx, Gy, per_pair);
    if (rc) return rc;
    if (!aligned8(ws)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (N == 0) return SPHBI_OK;
    if (T > 0 && (!ws || ws_bytes < sphbi_integrate_workspace(T))) {
        set_error("workspace too small (%zu < %zu)", ws_bytes, sphbi_integrate_workspace(T));
        return SPHBI_ENOWORKSPACE;
    }
    return integrate_run(kernel, opts, h, n_nodes, N, px, py, T, tri, nodal, (double *)ws, ws_bytes, offsets, tri_idx,
                         n_pairs, I, Gx, Gy, per_pair, stream);
}

int sphbi_integrate_quadrature(const sphbi_kernel *kernel, double h, int32_t n_nodes, int32_t n_gauss, int64_t N,
                               const double *px, const double *py, int64_t T, const double *tri,
                               const double *nodal, const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs,
                               double *I, double *Gx, double *Gy, void *stream) {
    sphbi_opts o;
    int rc = check_common(kernel, nullptr, &o, h, n_nodes, N, T, n_pairs);
    if (rc) return rc;
    if (n_gauss < 1 || n_gauss > SPHBI_MAX_GAUSS) {
        set_error("n_gauss must be in [1, %d]", SPHBI_MAX_GAUSS);
        return SPHBI_EINVAL;
    }
    if (N > 0 && (!px || !py || !offsets || !I || !Gx || !Gy)) { set_error("particle arrays are NULL"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && (!tri_idx || !tri || !nodal)) { set_error("pair/triangle arrays are NULL"); return SPHBI_EINVAL; }
    const void *ptrs[] = {px, py, tri, nodal, offsets, tri_idx, I, Gx, Gy};
    for (const void *p : ptrs)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    int deg = 0;
    const KArgs K = make_kargs(kernel, &deg);
    const int order = n_nodes == 1 ? 0 : (n_nodes == 3 ? 1 : 3);
    return launch_quadrature(order, deg, n_gauss, K, h, N, px, py, offsets, tri_idx, n_pairs, T, tri, nodal, I, Gx,
                             Gy, (hipStream_t)stream);
}

size_t sphbi_integrate_backward_workspace(int64_t T, int64_t n_pairs, int32_t n_nodes) {
    return backward_workspace(T > 0 ? T : 0, n_pairs > 0 ? n_pairs : 0, n_nodes == 10 ? 10 : (n_nodes == 3 ? 3 : 1));
}

int sphbi_integrate_backward(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, int32_t n_nodes,
                             int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                             const double *nodal, const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs,
                             const double *gI, const double *gGx, const double *gGy, double *dpx, double *dpy,
                             double *dtri, double *dnodal, void *ws, size_t ws_bytes, void *stream) {
    sphbi_opts o;
    int rc = check_common(kernel, opts, &o, h, n_nodes, N, T, n_pairs);
    if (rc) return rc;
    if (n_pairs > INT32_MAX) { set_error("more than 2^31-1 pairs"); return SPHBI_EUNSUPPORTED; }
    if (N > 0 && (!px || !py || !offsets || !gI || !gGx || !gGy || !dpx || !dpy)) {
        set_error("particle arrays are NULL");
        return SPHBI_EINVAL;
    }
    if (T > 0 && (!tri || !nodal || !dtri || !dnodal)) { set_error("triangle arrays are NULL"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && !tri_idx) { set_error("tri_idx is NULL"); return SPHBI_EINVAL; }
    const void *ptrs[] = {px, py, tri, nodal, offsets, tri_idx, gI, gGx, gGy, dpx, dpy, dtri, dnodal, ws};
    for (const void *p : ptrs)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    const size_t need = backward_workspace(T, n_pairs, n_nodes);
    if (!ws || ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return SPHBI_ENOWORKSPACE; }
    int deg = 0;
    const KArgs K = make_kargs(kernel, &deg);
    const int order = n_nodes == 1 ? 0 : (n_nodes == 3 ? 1 : 3);
    return launch_backward(order, deg, o.precision, o.tau_edge, K, h, N, px, py, offsets, tri_idx, n_pairs, T, tri,
                           nodal, gI, gGx, gGy, dpx, dpy, dtri, dnodal, ws, (hipStream_t)stream);
}

size_t sphbi_operator_workspace(int64_t N, int64_t T) { return operator_workspace(N, T); }

int sphbi_operator(const sphbi_kernel *kernel, const sphbi_opts *opts, int32_t op, double h, int32_t n_nodes,
                   int64_t N, const double *px, const double *py, const double *qa, const double *qb, int64_t T,
                   const double *tri, const double *fa, const double *fb, const int64_t *offsets,
                   const int32_t *tri_idx, int64_t n_pairs, double *out_a, double *out_b, void *ws, size_t ws_bytes,
                   void *stream) {
    if (op < SPHBI_OP_GRAD_DIFFERENCE || op > SPHBI_OP_NORMAL) { set_error("unknown operator %d", op); return SPHBI_EINVAL; }
    if (op == SPHBI_OP_NORMAL) n_nodes = 1;
    sphbi_opts o;
    int rc = check_common(kernel, opts, &o, h, n_nodes, N, T, n_pairs);
    if (rc) return rc;
    if (o.precision != SPHBI_FP64) { set_error("the operators run in FP64 only"); return SPHBI_EUNSUPPORTED; }
    const bool grad_form = op == SPHBI_OP_GRAD_DIFFERENCE || op == SPHBI_OP_GRAD_SYMMETRIC;
    if (N > 0 && (!px || !py || !offsets || !out_a || !out_b)) { set_error("particle arrays are NULL"); return SPHBI_EINVAL; }
    if (N > 0 && grad_form && (!qa || !qb)) { set_error("particle values qa/qb are NULL"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && (!tri_idx || !tri)) { set_error("pair/triangle arrays are NULL"); return SPHBI_EINVAL; }
    if (T > 0 && !tri) { set_error("triangle array is NULL"); return SPHBI_EINVAL; }
    if (T > 0 && op != SPHBI_OP_NORMAL && (!fa || !fb)) { set_error("nodal fields fa/fb are NULL"); return SPHBI_EINVAL; }
    const void *ptrs[] = {px, py, qa, qb, tri, fa, fb, offsets, tri_idx, out_a, out_b, ws};
    for (const void *p : ptrs)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (N == 0) return SPHBI_OK;
    const size_t need = operator_workspace(N, T);
    if (!ws || ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return SPHBI_ENOWORKSPACE; }
    int deg = 0;
    const KArgs K = make_kargs(kernel, &deg);
    const int order = n_nodes == 1 ? 0 : (n_nodes == 3 ? 1 : 3);
    return launch_operator(op, order, deg, K, h, N, px, py, qa, qb, offsets, tri_idx, n_pairs, T, tri, fa, fb, out_a,
                           out_b, ws, (hipStream_t)stream);
}

int sphbi_pressure_contact(const sphbi_kernel *kernel, const sphbi_opts *opts, double h, double rho0, int64_t N,
                           const double *px, const double *py, const double *p_particle,
                           const double *rho_particle, int64_t T, const double *tri, const int64_t *offsets,
                           const int32_t *tri_idx, int64_t n_pairs, const double *p_pair, double *ax, double *ay,
                           void *ws, size_t ws_bytes, void *stream) {
    sphbi_opts o;
    int rc = check_common(kernel, opts, &o, h, 1, N, T, n_pairs);
    if (rc) return rc;
    if (o.precision != SPHBI_FP64) { set_error("the pressure term runs in FP64 only"); return SPHBI_EUNSUPPORTED; }
    if (!(rho0 != 0.0) || !isfinite(rho0)) { set_error("rho0 must be finite and non-zero"); return SPHBI_EINVAL; }
    if (N > 0 && (!px || !py || !offsets || !p_particle || !rho_particle || !ax || !ay)) {
        set_error("particle arrays are NULL");
        return SPHBI_EINVAL;
    }
    if (n_pairs > 0 && (!tri_idx || !p_pair)) { set_error("pair arrays are NULL"); return SPHBI_EINVAL; }
    if (T > 0 && !tri) { set_error("triangle array is NULL"); return SPHBI_EINVAL; }
    const void *ptrs[] = {px, py, p_particle, rho_particle, tri, offsets, tri_idx, p_pair, ax, ay, ws};
    for (const void *p : ptrs)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (N == 0) return SPHBI_OK;
    const size_t need = operator_workspace(N, T);
    if (!ws || ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return SPHBI_ENOWORKSPACE; }
    int deg = 0;
    const KArgs K = make_kargs(kernel, &deg);
    return launch_pressure_contact(deg, K, h, rho0, N, px, py, p_particle, rho_particle, offsets, tri_idx, n_pairs, T,
                                   tri, p_pair, ax, ay, ws, (hipStream_t)stream);
}

// ----------------------------------------------------------------------------
// learned surrogate
// ----------------------------------------------------------------------------
static bool aligned(const void *p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

int sphbi_surrogate_features(double h, int64_t N, const double *px, const double *py, int64_t T, const double *tri,
                             const int64_t *offsets, const int32_t *tri_idx, int64_t n_pairs, float *feats,
                             float *rot, void *stream) {
    if (!(h > 0.0) || !isfinite(h)) { set_error("h must be positive and finite"); return SPHBI_EINVAL; }
    if (N < 0 || T < 0 || n_pairs < 0) { set_error("negative size"); return SPHBI_EINVAL; }
    if (N > kMaxItems || n_pairs > INT32_MAX) { set_error("too many particles or pairs in one call"); return SPHBI_EUNSUPPORTED; }
    if (N > 0 && (!px || !py || !offsets)) { set_error("particle arrays are NULL"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && (!tri_idx || !feats || !rot || (T > 0 && !tri))) { set_error("pair arrays are NULL"); return SPHBI_EINVAL; }
    const void *p8[] = {px, py, tri, offsets};
    for (const void *p : p8)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (!aligned(feats, 4) || !aligned(rot, 4) || !aligned(tri_idx, 4)) { set_error("arrays must be 4-byte aligned"); return SPHBI_EINVAL; }
    return surrogate_features(h, N, px, py, T, tri, offsets, tri_idx, n_pairs, feats, rot, (hipStream_t)stream);
}

int sphbi_surrogate_targets(int64_t n_pairs, double h, const double *per_pair, const float *rot, const float *mean,
                            const float *stdev, float *targets, void *stream) {
    if (n_pairs < 0 || !(h > 0.0) || !isfinite(h)) { set_error("invalid size or h"); return SPHBI_EINVAL; }
    if (n_pairs > INT32_MAX) { set_error("more than 2^31-1 pairs in one call"); return SPHBI_EUNSUPPORTED; }
    if (!mean || !stdev) { set_error("NULL statistics"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && (!per_pair || !rot || !targets)) { set_error("NULL array"); return SPHBI_EINVAL; }
    if (!aligned8(per_pair) || !aligned(rot, 4) || !aligned(targets, 4)) { set_error("misaligned array"); return SPHBI_EINVAL; }
    SurrogateStats st;
    for (int k = 0; k < 3; ++k) {
        if (!(stdev[k] > 0.0f)) { set_error("stdev must be positive"); return SPHBI_EINVAL; }
        st.mean[k] = mean[k];
        st.stdev[k] = stdev[k];
    }
    st.fmax = 0.0f;
    return surrogate_targets(n_pairs, h, per_pair, rot, st, targets, (hipStream_t)stream);
}

size_t sphbi_mlp_workspace(int64_t B) { return B < 0 ? 0 : mlp_workspace(B); }

static int check_batch(int64_t B, const void *ws, size_t ws_bytes) {
    if (B < 0 || B > ((int64_t)1 << 30)) { set_error("batch size %lld out of range", (long long)B); return SPHBI_EINVAL; }
    const size_t need = mlp_workspace(B);
    if (!ws || ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return SPHBI_ENOWORKSPACE; }
    if (!aligned(ws, 256)) { set_error("workspace must be 256-byte aligned"); return SPHBI_EINVAL; }
    return SPHBI_OK;
}

int sphbi_mlp_forward(const float *params, int64_t B, const float *feats, float *out, void *ws, size_t ws_bytes,
                      void *stream) {
    if (B == 0) return SPHBI_OK;
    int rc = check_batch(B, ws, ws_bytes);
    if (rc) return rc;
    if (!params || !feats || !out) { set_error("NULL array"); return SPHBI_EINVAL; }
    if (!aligned(params, 4) || !aligned(feats, 4) || !aligned(out, 4)) { set_error("arrays must be 4-byte aligned"); return SPHBI_EINVAL; }
    return mlp_forward(params, B, feats, out, ws, (hipStream_t)stream);
}

int sphbi_mlp_loss_grad(const float *params, int64_t B, const float *feats, const float *targets, const float *scale,
                        float lam, float *loss, float *grad, void *ws, size_t ws_bytes, void *stream) {
    if (B <= 0) { set_error("empty batch"); return SPHBI_EINVAL; }
    int rc = check_batch(B, ws, ws_bytes);
    if (rc) return rc;
    if (!params || !feats || !targets || !scale || !loss || !grad) { set_error("NULL array"); return SPHBI_EINVAL; }
    if (!(lam >= 0.0f) || !isfinite(lam)) { set_error("lam must be finite and >= 0"); return SPHBI_EINVAL; }
    const void *p4[] = {params, feats, targets, loss, grad};
    for (const void *p : p4)
        if (!aligned(p, 4)) { set_error("arrays must be 4-byte aligned"); return SPHBI_EINVAL; }
    return mlp_loss_grad(params, B, feats, targets, scale, lam, loss, grad, ws, (hipStream_t)stream);
}

int sphbi_adam_step(float *params, float *m, float *v, const float *grad, int64_t n, double lr, double beta1,
                    double beta2, double eps, int64_t step, void *stream) {
    if (n < 0 || step < 1) { set_error("n must be >= 0 and step >= 1"); return SPHBI_EINVAL; }
    if (!(beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0 && isfinite(lr))) {
        set_error("invalid Adam hyper-parameters");
        return SPHBI_EINVAL;
    }
    if (n > 0 && (!params || !m || !v || !grad)) { set_error("NULL array"); return SPHBI_EINVAL; }
    return adam_step(params, m, v, grad, n, lr, beta1, beta2, eps, step, (hipStream_t)stream);
}

size_t sphbi_surrogate_model_bytes(void) { return surrogate_model_bytes(); }

int sphbi_surrogate_pack(const float *params, const float *mean, const float *stdev, float fmax, void *model,
                         void *stream) {
    if (!params || !mean || !stdev || !model) { set_error("NULL array"); return SPHBI_EINVAL; }
    if (!aligned(model, 16) || !aligned(params, 4)) { set_error("model must be 16-byte aligned"); return SPHBI_EINVAL; }
    SurrogateStats st;
    for (int k = 0; k < 3; ++k) {
        st.mean[k] = mean[k];
        st.stdev[k] = stdev[k];
    }
    st.fmax = fmax;
    return surrogate_pack(params, st, model, (hipStream_t)stream);
}

size_t sphbi_surrogate_workspace(int64_t T, int64_t n_pairs) {
    return (T < 0 || n_pairs < 0) ? 0 : surrogate_workspace(T, n_pairs);
}

int sphbi_surrogate_integrate(const sphbi_kernel *kernel, double h, int64_t N, const double *px, const double *py,
                              int64_t T, const double *tri, const double *nodal, const int64_t *offsets,
                              const int32_t *tri_idx, int64_t n_pairs, const void *model, float threshold, double *I,
                              double *Gx, double *Gy, double *per_pair, uint8_t *flags, int64_t *n_flagged, void *ws,
                              size_t ws_bytes, void *stream) {
    int rc = validate_kernel(kernel);
    if (rc) return rc;
    if (!(h > 0.0) || !isfinite(h)) { set_error("h must be positive and finite"); return SPHBI_EINVAL; }
    if (N < 0 || T < 0 || n_pairs < 0) { set_error("negative size"); return SPHBI_EINVAL; }
    if (N > kMaxItems || T > kMaxItems || n_pairs > INT32_MAX) {
        set_error("too many particles, triangles or pairs in one call");
        return SPHBI_EUNSUPPORTED;
    }
    if (N > 0 && (!px || !py || !offsets || !I || !Gx || !Gy || !n_flagged || !model)) { set_error("NULL array"); return SPHBI_EINVAL; }
    if (n_pairs > 0 && (!tri_idx || !flags || !tri || !nodal)) { set_error("pair/triangle arrays are NULL"); return SPHBI_EINVAL; }
    const void *p8[] = {px, py, tri, nodal, offsets, I, Gx, Gy, per_pair, n_flagged};
    for (const void *p : p8)
        if (!aligned8(p)) { set_error("arrays must be 8-byte aligned"); return SPHBI_EINVAL; }
    if (!aligned(model, 16) || !aligned(ws, 256)) { set_error("model/workspace misaligned"); return SPHBI_EINVAL; }
    if (N == 0) return SPHBI_OK;
    const size_t need = surrogate_workspace(T, n_pairs);
    if (!ws || ws_bytes < need) { set_error("workspace too small (%zu < %zu)", ws_bytes, need); return SPHBI_ENOWORKSPACE; }
    int deg = 0;
    const KArgs K = make_kargs(kernel, &deg);
    return surrogate_integrate(K, deg, h, N, px, py, T, tri, nodal, offsets, tri_idx, n_pairs, model, threshold, I, Gx,
                               Gy, per_pair, flags, n_flagged, ws, (hipStream_t)stream);
}

}  // extern "C"

