// Setup on the device (Section 3.1), for meshes whose nodes move between
// searches: element AABB and OBB (Sections 3.1.1, 3.1.2, 4.1, 4.2) and the
// local map (Section 3.1.3), recomputed from the device copy of the nodes.
//
// Every quantity is computed with the operations of the host setup in the
// same order, and this file is compiled without floating-point contraction,
// so the boxes and the map equal those of fpts_setup on the same nodes bit
// for bit.  One wave per element: sums whose order fixes the rounding run
// in one lane; the Chebyshev-grid evaluations of the bounds run across
// lanes (each lane one grid point, the reduction is a min/max).
#include <cmath>
#include <vector>

#include "fpts_internal.hpp"

namespace fpts {
namespace {

constexpr int kLanes = 64;

// std::min / std::max semantics (first argument on ties)
__device__ __forceinline__ double mn(double a, double b) { return (b < a) ? b : a; }
__device__ __forceinline__ double mx(double a, double b) { return (a < b) ? b : a; }

__device__ __forceinline__ void wave_minmax(double &lo, double &hi)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        lo = mn(lo, __shfl_xor(lo, o));
        hi = mx(hi, __shfl_xor(hi, o));
    }
}

// Bound of u(r) = sum_i u_i phi_i(r) (eqs. eq_1D_bound_final_1/2): linear
// Legendre part removed, basis bounds at the M Chebyshev points.  u in LDS,
// sc: LDS scratch of the wave.  Result uniform over the wave.
__device__ void bound1_w(const BoundTables &T, const double *u, double *sc, int lane,
                         double &lo, double &hi)
{
    const int N = T.N, M = T.M;
    if (lane == 0) {
        double a0 = 0.0, a1 = 0.0;
        for (int i = 0; i < N; ++i) {
            a0 += u[i] * T.mom0[i];
            a1 += u[i] * T.mom1[i];
        }
        sc[0] = a0 * 0.5;
        sc[1] = a1 * 1.5;
    }
    __syncthreads();
    const double a0 = sc[0], a1 = sc[1];
    double l = INFINITY, h = -INFINITY;
    if (lane < M) {
        const int j = lane;
        l = a0 + a1 * T.eta[j];
        h = l;
        for (int i = 0; i < N; ++i) {
            const double w = u[i] - (a0 + a1 * T.z[i]);
            const double x = w * T.vlo[i * M + j], y = w * T.vhi[i * M + j];
            l += mn(x, y);
            h += mx(x, y);
        }
    }
    wave_minmax(l, h);
    lo = l;
    hi = h;
    __syncthreads();
}

// Bound of u(r,s) = sum_ij u_ij phi_i(r) phi_j(s), u indexed i + N j (eqs.
// eq_2D_function_bound_1/2), bilinear Legendre part removed.  w: LDS [N*N].
__device__ void bound2_w(const BoundTables &T, const double *u, double *w, double *sc,
                         int lane, double &lo, double &hi)
{
    const int N = T.N, M = T.M;
    if (lane == 0) {
        double a00 = 0, a10 = 0, a01 = 0, a11 = 0;
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const double x = u[i + N * j];
                a00 += x * T.mom0[i] * T.mom0[j];
                a10 += x * T.mom1[i] * T.mom0[j];
                a01 += x * T.mom0[i] * T.mom1[j];
                a11 += x * T.mom1[i] * T.mom1[j];
            }
        sc[0] = a00 * 0.25;
        sc[1] = a10 * 0.75;
        sc[2] = a01 * 0.75;
        sc[3] = a11 * 2.25;
    }
    __syncthreads();
    const double a00 = sc[0], a10 = sc[1], a01 = sc[2], a11 = sc[3];
    for (int idx = lane; idx < N * N; idx += kLanes) {
        const int i = idx % N, j = idx / N;
        w[idx] = u[idx] - (a00 + a10 * T.z[i] + a01 * T.z[j] + a11 * T.z[i] * T.z[j]);
    }
    __syncthreads();
    double l = INFINITY, h = -INFINITY;
    for (int gp = lane; gp < M * M; gp += kLanes) {
        const int k = gp % M, ll = gp / M;
        const double b = a00 + a10 * T.eta[k] + a01 * T.eta[ll] + a11 * T.eta[k] * T.eta[ll];
        double sl = b, sh = b;
        for (int i = 0; i < N; ++i) {
            const double ulo = T.vlo[i * M + k], uhi = T.vhi[i * M + k];
            for (int j = 0; j < N; ++j) {
                const double x = w[i + N * j];
                const double vlo = T.vlo[j * M + ll], vhi = T.vhi[j * M + ll];
                const double p1 = ulo * vlo, p2 = ulo * vhi, p3 = uhi * vlo, p4 = uhi * vhi;
                const double pn = mn(mn(p1, p2), mn(p3, p4));
                const double px = mx(mx(p1, p2), mx(p3, p4));
                sl += x >= 0.0 ? x * pn : x * px;
                sh += x >= 0.0 ? x * px : x * pn;
            }
        }
        l = mn(l, sl);
        h = mx(h, sh);
    }
    wave_minmax(l, h);
    lo = l;
    hi = h;
    __syncthreads();
}

// Bound of one coordinate function f[NP] (LDS): the edges of a quad, the
// faces of a hex, the whole patch of a surface quad, the whole curve of a
// line element.
__device__ void bound_fun_w(const BoundTables &T, int D, int R, const double *f, double *buf,
                            double *w, double *sc, int lane, double &lo, double &hi)
{
    const int N = T.N;
    double a, b;
    lo = INFINITY;
    hi = -INFINITY;
    if (R == 2 && D == 2) {
        for (int e = 0; e < 2; ++e) {
            const int q = e ? N - 1 : 0;
            for (int i = lane; i < N; i += kLanes) buf[i] = f[i + N * q];
            __syncthreads();
            bound1_w(T, buf, sc, lane, a, b);
            lo = mn(lo, a);
            hi = mx(hi, b);
            for (int j = lane; j < N; j += kLanes) buf[j] = f[q + N * j];
            __syncthreads();
            bound1_w(T, buf, sc, lane, a, b);
            lo = mn(lo, a);
            hi = mx(hi, b);
        }
    } else if (R == 3) {
        for (int e = 0; e < 2; ++e) {
            const int q = e ? N - 1 : 0;
            for (int t = 0; t < 3; ++t) {
                for (int idx = lane; idx < N * N; idx += kLanes) {
                    const int x0 = idx % N, x1 = idx / N;
                    buf[idx] = t == 0   ? f[x0 + N * (x1 + N * q)]
                               : t == 1 ? f[x0 + N * (q + N * x1)]
                                        : f[q + N * (x0 + N * x1)];
                }
                __syncthreads();
                bound2_w(T, buf, w, sc, lane, a, b);
                lo = mn(lo, a);
                hi = mx(hi, b);
            }
        }
    } else if (R == 2) {
        bound2_w(T, f, w, sc, lane, a, b);
        lo = mn(lo, a);
        hi = mx(hi, b);
    } else {
        bound1_w(T, f, sc, lane, a, b);
        lo = mn(lo, a);
        hi = mx(hi, b);
    }
}

// Thin-extent rule (manifolds; reference: the smallest other extent, the
// largest for lines) and expansion by tol of the extent in total.
__device__ void finish_d(int D, int R, double tol, double *lo, double *hi, const double *len)
{
    double L[3];
    for (int d = 0; d < D; ++d) L[d] = hi[d] - lo[d];
    if (R < D) {
        double P[3];
        for (int d = 0; d < D; ++d) P[d] = L[d] * len[d];
        for (int d = 0; d < D; ++d) {
            double ref = R == 1 ? 0.0 : INFINITY;
            for (int q = 0; q < D; ++q)
                if (q != d) ref = R == 1 ? mx(ref, P[q]) : mn(ref, P[q]);
            const double need = tol * ref / len[d];
            if (L[d] < need) {
                const double c = 0.5 * (lo[d] + hi[d]);
                lo[d] = c - 0.5 * need;
                hi[d] = c + 0.5 * need;
                L[d] = need;
            }
        }
    }
    for (int d = 0; d < D; ++d) {
        lo[d] -= 0.5 * tol * L[d];
        hi[d] += 0.5 * tol * L[d];
    }
}

__device__ bool invert_d(int D, const double *A, double *I)
{
    if (D == 2) {
        const double det = A[0] * A[3] - A[1] * A[2];
        if (!(det != 0.0) || !isfinite(det)) return false;
        I[0] = A[3] / det;
        I[1] = -A[1] / det;
        I[2] = -A[2] / det;
        I[3] = A[0] / det;
        return true;
    }
    const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8],
                 c02 = A[3] * A[7] - A[4] * A[6];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(det != 0.0) || !isfinite(det)) return false;
    const double id = 1.0 / det;
    I[0] = c00 * id;
    I[3] = c01 * id;
    I[6] = c02 * id;
    I[1] = (A[2] * A[7] - A[1] * A[8]) * id;
    I[4] = (A[0] * A[8] - A[2] * A[6]) * id;
    I[7] = (A[1] * A[6] - A[0] * A[7]) * id;
    I[2] = (A[1] * A[5] - A[2] * A[4]) * id;
    I[5] = (A[2] * A[3] - A[0] * A[5]) * id;
    I[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    return true;
}

// AABB and OBB record (lo, hi, OBB centre, OBB inverse transform) and
// centre of every element; one wave per element.
__global__ __launch_bounds__(kLanes) void k_elem_boxes(const BoundTables *Tg, const double *nodes,
                                                      int64_t nel, int D, int R, double tol,
                                                      double *box, double *xc_out)
{
    extern __shared__ double lds[];
    const BoundTables &T = *Tg;
    const int N = T.N, NP = (R == 3) ? N * N * N : (R == 2) ? N * N : N, W = 3 * D + D * D;
    const int lane = threadIdx.x;
    double *xe = lds;              // [D][NP]
    double *f = xe + D * NP;       // [NP]
    double *buf = f + NP;          // [N*N]
    double *w = buf + N * N;       // [N*N]
    double *sc = w + N * N;        // scratch (16)
    for (int64_t e = blockIdx.x; e < nel; e += gridDim.x) {
        for (int idx = lane; idx < D * NP; idx += kLanes) xe[idx] = nodes[e * D * NP + idx];
        __syncthreads();
        double lo[3], hi[3], one[3] = {1, 1, 1};
        for (int c = 0; c < D; ++c)
            bound_fun_w(T, D, R, xe + c * NP, buf, w, sc, lane, lo[c], hi[c]);
        finish_d(D, R, tol, lo, hi, one);
        // centre and centre Jacobian, in one lane (summation order)
        if (lane == 0) {
            double xc[3] = {0, 0, 0}, G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
            for (int idx = 0; idx < NP; ++idx) {
                const int ii = idx % N, jj = (idx / N) % N, kk = idx / (N * N);
                double b0 = T.v0[ii] * T.v0[jj], br = T.d0[ii] * T.v0[jj],
                       bs = T.v0[ii] * T.d0[jj], bt = 0.0;
                if (R == 1) {
                    b0 = T.v0[ii];
                    br = T.d0[ii];
                    bs = 0.0;
                }
                if (R == 3) {
                    bt = b0 * T.d0[kk];
                    b0 *= T.v0[kk];
                    br *= T.v0[kk];
                    bs *= T.v0[kk];
                }
                for (int c = 0; c < D; ++c) {
                    const double xv = xe[c * NP + idx];
                    xc[c] += xv * b0;
                    G[c][0] += xv * br;
                    G[c][1] += xv * bs;
                    if (R == 3) G[c][2] += xv * bt;
                }
            }
            for (int c = 0; c < 3; ++c) {
                sc[4 + c] = xc[c];
                for (int a = 0; a < 3; ++a) sc[7 + 3 * c + a] = G[c][a];
            }
        }
        __syncthreads();
        double xc[3], G[3][3];
        for (int c = 0; c < 3; ++c) {
            xc[c] = sc[4 + c];
            for (int a = 0; a < 3; ++a) G[c][a] = sc[7 + 3 * c + a];
        }
        __syncthreads();
        double Jc[9] = {0}, Ji[9] = {0}, len[3] = {1, 1, 1};
        if (R == D) {
            for (int a = 0; a < D; ++a)
                for (int b = 0; b < D; ++b) Jc[a * D + b] = G[a][b];
        } else if (R == 1) {
            rodrigues_frame(D, G[0][0], G[1][0], D == 3 ? G[2][0] : 0.0, Jc);
        } else {
            const double t1[3] = {G[0][0], G[1][0], G[2][0]}, t2[3] = {G[0][1], G[1][1], G[2][1]};
            const double n[3] = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2],
                                 t1[0] * t2[1] - t1[1] * t2[0]};
            const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            for (int c = 0; c < 3; ++c) {
                Jc[c * 3 + 0] = t1[c];
                Jc[c * 3 + 1] = t2[c];
                Jc[c * 3 + 2] = nn > 0.0 ? n[c] / nn : 0.0;
            }
            len[0] = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
            len[1] = sqrt(t2[0] * t2[0] + t2[1] * t2[1] + t2[2] * t2[2]);
        }
        double *rec = box + e * W;
        const bool inv = invert_d(D, Jc, Ji);
        double tl[3], th[3];
        if (inv) {
            for (int c = 0; c < D; ++c) {
                for (int idx = lane; idx < NP; idx += kLanes) {
                    double s = 0.0;
                    for (int q = 0; q < D; ++q) s += Ji[c * D + q] * (xe[q * NP + idx] - xc[q]);
                    f[idx] = s;
                }
                __syncthreads();
                bound_fun_w(T, D, R, f, buf, w, sc, lane, tl[c], th[c]);
            }
            finish_d(D, R, tol, tl, th, len);
        }
        if (lane == 0) {
            for (int c = 0; c < D; ++c) {
                rec[c] = lo[c];
                rec[D + c] = hi[c];
                xc_out[e * D + c] = xc[c];
            }
            double *oc = rec + 2 * D, *oA = rec + 3 * D;
            if (!inv) {
                for (int c = 0; c < D; ++c) oc[c] = xc[c];
                for (int a = 0; a < D * D; ++a) oA[a] = 0.0;
            } else {
                for (int a = 0; a < D; ++a) {
                    const double half = 0.5 * (th[a] - tl[a]);
                    for (int b = 0; b < D; ++b) oA[a * D + b] = Ji[a * D + b] / half;
                }
                for (int c = 0; c < D; ++c) {
                    double s = xc[c];
                    for (int q = 0; q < D; ++q) s += Jc[c * D + q] * 0.5 * (th[q] + tl[q]);
                    oc[c] = s;
                }
            }
        }
        __syncthreads();
    }
}

// Per block: min of the AABB lows and max of the highs over its elements.
__global__ __launch_bounds__(256) void k_union(const double *box, int64_t nel, int D,
                                              double *part)
{
    __shared__ double red[256];
    const int W = 3 * D + D * D;
    for (int q = 0; q < 2 * D; ++q) {
        const bool low = q < D;
        double v = low ? INFINITY : -INFINITY;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nel;
             e += (int64_t)gridDim.x * blockDim.x) {
            const double x = box[e * W + q];
            v = low ? mn(v, x) : mx(v, x);
        }
        red[threadIdx.x] = v;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o)
                red[threadIdx.x] = low ? mn(red[threadIdx.x], red[threadIdx.x + o])
                                       : mx(red[threadIdx.x], red[threadIdx.x + o]);
            __syncthreads();
        }
        if (threadIdx.x == 0) part[blockIdx.x * 2 * D + q] = red[0];
        __syncthreads();
    }
}

struct MapView {
    double lo[3], del[3];
    int NL, D;
};

__device__ __forceinline__ int cell_coord_d(const MapView &v, int d, double x)
{
    double t = floor((x - v.lo[d]) / v.del[d]);
    if (t < 0.0) t = 0.0;
    if (t > v.NL - 1) t = v.NL - 1;
    return (int)t;
}

// pass 0: count the cells spanned by each element's AABB corners; pass 1:
// write the element into each of them
__global__ __launch_bounds__(256) void k_map(MapView v, const double *box, int64_t nel, int pass,
                                            int *cnt, const int *off, int *fill, int *cell_el)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nel) return;
    const int D = v.D, W = 3 * D + D * D;
    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) {
        c0[d] = cell_coord_d(v, d, box[e * W + d]);
        c1[d] = cell_coord_d(v, d, box[e * W + D + d]);
    }
    const int64_t NL = v.NL;
    for (int k = c0[2]; k <= c1[2]; ++k)
        for (int j = c0[1]; j <= c1[1]; ++j)
            for (int i = c0[0]; i <= c1[0]; ++i) {
                const int64_t c = i + NL * (j + NL * k);
                if (pass == 0) atomicAdd(&cnt[c], 1);
                else cell_el[off[c] + atomicAdd(&fill[c], 1)] = (int)e;
            }
}

// each cell's element list in ascending id (the host registers elements in
// ascending order)
__global__ __launch_bounds__(256) void k_map_sort(const int *off, int64_t ncell, int *cell_el)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int b = off[c], n = off[c + 1] - b;
    int *a = cell_el + b;
    for (int i = 1; i < n; ++i) {
        const int x = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > x) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = x;
    }
}

template <typename T>
struct DevBuf {
    T *p = nullptr;
    ~DevBuf() { (void)hipFree(p); }
    bool alloc(size_t n) { return hipMalloc(&p, sizeof(T) * std::max<size_t>(n, 1)) == hipSuccess; }
};

}  // namespace

int device_setup(fpts_mesh *m, hipStream_t s)
{
    const int D = m->D, R = m->R, N = m->N, NP = m->NP, W = box_words(D);
    BoundTables bt;
    bound_tables(m, &bt);
    DevBuf<BoundTables> dt;
    if (!dt.alloc(1)) return FPTS_ENOMEM;
    if (hipMemcpyAsync(dt.p, &bt, sizeof(bt), hipMemcpyHostToDevice, s) != hipSuccess)
        return FPTS_EDEVICE;
    // boxes and centres
    const size_t lds = sizeof(double) * (D * NP + NP + 2 * N * N + 16);
    const int grid = (int)std::min<int64_t>(m->nel, (int64_t)m->cus * 16);
    hipLaunchKernelGGL(k_elem_boxes, dim3(grid), dim3(kLanes), lds, s, dt.p, m->d_nodes,
                       (int64_t)m->nel, D, R, m->p.bbox_tol, m->d_box, m->d_xc);
    if (hipGetLastError() != hipSuccess) return FPTS_EDEVICE;
    // union box
    const int ublocks = (int)std::min<int64_t>((m->nel + 255) / 256, 1024);
    DevBuf<double> part;
    if (!part.alloc((size_t)ublocks * 2 * D)) return FPTS_ENOMEM;
    hipLaunchKernelGGL(k_union, dim3(ublocks), dim3(256), 0, s, m->d_box, (int64_t)m->nel, D,
                       part.p);
    std::vector<double> hp((size_t)ublocks * 2 * D);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(hp.data(), part.p, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FPTS_EDEVICE;
    for (int d = 0; d < D; ++d) {
        m->hlo[d] = INFINITY;
        m->hhi[d] = -INFINITY;
    }
    for (int b = 0; b < ublocks; ++b)
        for (int d = 0; d < D; ++d) {
            m->hlo[d] = std::min(m->hlo[d], hp[(size_t)b * 2 * D + d]);
            m->hhi[d] = std::max(m->hhi[d], hp[(size_t)b * 2 * D + D + d]);
        }
    for (int d = 0; d < D; ++d)
        if (!std::isfinite(m->hlo[d]) || !std::isfinite(m->hhi[d]) || !(m->hhi[d] > m->hlo[d]))
            return FPTS_EINVAL;
    // the map resolution is the mesh's (hash_n or the default, unchanged)
    const int NL = m->NL;
    for (int d = 0; d < D; ++d) m->hdel[d] = (m->hhi[d] - m->hlo[d]) / NL;
    int64_t ncell = 1;
    for (int d = 0; d < D; ++d) ncell *= NL;
    MapView v;
    for (int d = 0; d < 3; ++d) {
        v.lo[d] = d < D ? m->hlo[d] : 0.0;
        v.del[d] = d < D ? m->hdel[d] : 1.0;
    }
    v.NL = NL;
    v.D = D;
    DevBuf<int> cnt, fill, tmp;
    const int64_t tb = scan_tmp_blocks(ncell);
    if (!cnt.alloc(ncell + 1) || !fill.alloc(ncell) || !tmp.alloc(tb)) return FPTS_ENOMEM;
    const int eg = (int)((m->nel + 255) / 256);
    if (launch_fill_i32(cnt.p, ncell, 0, s) != hipSuccess ||
        launch_fill_i32(fill.p, ncell, 0, s) != hipSuccess)
        return FPTS_EDEVICE;
    hipLaunchKernelGGL(k_map, dim3(eg), dim3(256), 0, s, v, m->d_box, (int64_t)m->nel, 0, cnt.p,
                       nullptr, nullptr, nullptr);
    if (hipGetLastError() != hipSuccess ||
        launch_exclusive_scan(cnt.p, m->d_cell_off, ncell, 1, tmp.p, tb, s) != hipSuccess)
        return FPTS_EDEVICE;
    m->cell_off.resize(ncell + 1);
    if (hipMemcpyAsync(m->cell_off.data(), m->d_cell_off, sizeof(int) * (ncell + 1),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FPTS_EDEVICE;
    const int64_t nnz = m->cell_off[ncell];
    if (nnz > (int64_t)m->cell_el.size()) {
        int *p = nullptr;
        if (hipMalloc(&p, sizeof(int) * nnz) != hipSuccess) return FPTS_ENOMEM;
        (void)hipFree(m->d_cell_el);
        m->d_cell_el = p;
    }
    m->cell_el.resize(std::max<int64_t>(nnz, 1));
    hipLaunchKernelGGL(k_map, dim3(eg), dim3(256), 0, s, v, m->d_box, (int64_t)m->nel, 1, nullptr,
                       m->d_cell_off, fill.p, m->d_cell_el);
    hipLaunchKernelGGL(k_map_sort, dim3((int)((ncell + 255) / 256)), dim3(256), 0, s,
                       m->d_cell_off, ncell, m->d_cell_el);
    m->max_cell = 0;
    for (int64_t c = 0; c < ncell; ++c)
        m->max_cell = std::max(m->max_cell, m->cell_off[c + 1] - m->cell_off[c]);
    // host copies of the products (fpts_get_boxes, fpts_get_hash, workspace sizes)
    m->box.resize((size_t)m->nel * W);
    m->xc.resize((size_t)m->nel * D);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(m->cell_el.data(), m->d_cell_el, sizeof(int) * nnz, hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipMemcpyAsync(m->box.data(), m->d_box, sizeof(double) * m->box.size(),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(m->xc.data(), m->d_xc, sizeof(double) * m->xc.size(),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FPTS_EDEVICE;
    return FPTS_OK;
}

}  // namespace fpts
