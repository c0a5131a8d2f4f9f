// HIP kernels of libscpl.so for gfx950 (MI355X): SCPL video retargeting.
//
// Method: "Fast Video Retargeting Based on Seam Carving with Parental
// Labeling" (arXiv 1903.03180).  Stage map:
//   luma_kernel        colour -> 8-bit luma (the paper does not say which
//                      channel feeds the energy; BT.601 luma is used)
//   seg_window_kernel  energy (Sec. 3.3) + ASDE moments (eqs. 7-8) for a
//                      window of candidate frames of one buffer (Sec. 3.2)
//   energy_kernel      uniform energy of a buffer (Sec. 3.2): mean of the
//                      frames' motion-aware energies, read through the
//                      buffer's column map so frames are never recopied
//   dp_kernel          cumulative energy, eq. (4), with the row-0 parent
//                      label carried along the argmin path (Sec. 3.1)
//   borg_kernel        band origins for the two-level backtrack
//   select_kernel      per-parent least child (eq. 6), top-k, band jumps
//   fill_kernel        seams inside each band; buffer mask
//   compact_kernel     removes k_iter seams from the column map in one pass
//   gather_kernel      carved output frames and masks
#include "scpl_internal.h"

namespace scpl {

namespace {

constexpr int kInf = 0x7fffffff;

__device__ __forceinline__ int job_width(const Job &J, int r) { return r < J.logcap ? J.log[4 * r] : J.Wt; }

// A column-map entry, kept inside [0, W) so that no address can leave the
// frame even if the map were corrupt (the parity tests would catch that).
__device__ __forceinline__ int mcol(const int16_t *m, int j, int W) { return min(max((int)m[j], 0), W - 1); }

// |Gx| + |Gy| of the 3x3 Sobel operator from nine pixels p[row][col].
__device__ __forceinline__ int sobel9(int a0, int a1, int a2, int b0, int b2, int c0, int c1, int c2)
{
    int gx = (a2 + 2 * b2 + c2) - (a0 + 2 * b0 + c0);
    int gy = (c0 + 2 * c1 + c2) - (a0 + 2 * a1 + a2);
    return abs(gx) + abs(gy);
}

__device__ __forceinline__ uint32_t isqrt_u64(uint64_t q)
{
    uint64_t r = (uint64_t)sqrt((double)q);
    while (r * r > q) --r;
    while ((r + 1) * (r + 1) <= q) ++r;
    return (uint32_t)r;
}

// Exclusive prefix sum of v over the block (blockDim.x a multiple of 64,
// at most 1024).  tmp holds 16 ints.  Returns the block total in *total.
__device__ int block_exclusive_scan(int v, int *tmp, int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) tmp[wid] = x;
    __syncthreads();
    if (wid == 0) {
        int w = lane < nw ? tmp[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            int y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < 16) tmp[lane] = w;  // inclusive wave totals
    }
    __syncthreads();
    *total = tmp[nw - 1];
    int base = wid > 0 ? tmp[wid - 1] : 0;
    int r = base + x - v;
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- luma

__global__ __launch_bounds__(256) void luma_vec_kernel(const uint8_t *__restrict__ rgb, uint8_t *__restrict__ y,
                                                       int64_t npx)
{
    const int64_t p0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
    if (p0 >= npx) return;
    if (p0 + 16 <= npx) {
        const uint4 *src = reinterpret_cast<const uint4 *>(rgb + p0 * 3);
        uint4 a = src[0], b = src[1], c = src[2];
        const uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
        uint32_t o[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int k0 = 3 * q, k1 = 3 * q + 1, k2 = 3 * q + 2;
            const uint32_t R = (w[k0 >> 2] >> (8 * (k0 & 3))) & 255u;
            const uint32_t G = (w[k1 >> 2] >> (8 * (k1 & 3))) & 255u;
            const uint32_t B = (w[k2 >> 2] >> (8 * (k2 & 3))) & 255u;
            const uint32_t v = (77u * R + 150u * G + 29u * B + 128u) >> 8;
            o[q >> 2] |= v << (8 * (q & 3));
        }
        *reinterpret_cast<uint4 *>(y + p0) = make_uint4(o[0], o[1], o[2], o[3]);
    } else {
        for (int64_t p = p0; p < npx; ++p)
            y[p] = (uint8_t)((77u * rgb[3 * p] + 150u * rgb[3 * p + 1] + 29u * rgb[3 * p + 2] + 128u) >> 8);
    }
}

__global__ __launch_bounds__(256) void luma_scalar_kernel(const uint8_t *__restrict__ rgb, uint8_t *__restrict__ y,
                                                          int64_t npx)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < npx) y[p] = (uint8_t)((77u * rgb[3 * p] + 150u * rgb[3 * p + 1] + 29u * rgb[3 * p + 2] + 128u) >> 8);
}

// ------------------------------------------------------- ASDE window scan
//
// One thread per pixel of the original frame.  For a buffer starting at t0
// whose moments S1 = sum e, S2 = sum e^2 cover frames [t0, tb), frames
// [tb, te) are appended one at a time; after each one the per-pixel
// floor(sqrt(n S2 - S1^2)) (n times the population deviation of eq. 8) is
// summed into sout[t - tb].  The host then decides every candidate in order
// (eq. 9) and discards the tail after the first rejection.

__global__ __launch_bounds__(256) void seg_window_kernel(SegArgs a)
{
    __shared__ unsigned long long part[kSegWindow];
    const int tid = threadIdx.x;
    if (tid < kSegWindow) part[tid] = 0;
    __syncthreads();
    const int64_t HW = (int64_t)a.H * a.W;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    const bool valid = p < HW;
    const int i = valid ? (int)(p / a.W) : 0;
    const int j = valid ? (int)(p - (int64_t)i * a.W) : 0;
    const int im = max(i - 1, 0), ip = min(i + 1, a.H - 1), jm = max(j - 1, 0), jp = min(j + 1, a.W - 1);
    const int oa = im * a.W, ob = i * a.W, oc = ip * a.W;
    uint32_t s1 = 0;
    uint64_t s2 = 0;
    if (valid) {
        if (a.init) {
            const uint8_t *f = a.luma + (size_t)a.t0 * HW;
            const int g = sobel9(f[oa + jm], f[oa + j], f[oa + jp], f[ob + jm], f[ob + jp], f[oc + jm], f[oc + j],
                                 f[oc + jp]);
            uint32_t e = (uint32_t)g;
            if (a.mode == 1) e = 2u * g + (a.t0 > 0 ? 18u * (uint32_t)abs((int)f[p] - (int)f[p - HW]) : 0u);
            s1 = e;
            s2 = (uint64_t)e * e;
        } else {
            s1 = a.s1[p];
            s2 = a.s2[p];
        }
    }
    for (int t = a.tb; t < a.te; ++t) {
        unsigned long long v = 0;
        if (valid) {
            const uint8_t *f = a.luma + (size_t)t * HW;
            const int g = sobel9(f[oa + jm], f[oa + j], f[oa + jp], f[ob + jm], f[ob + jp], f[oc + jm], f[oc + j],
                                 f[oc + jp]);
            uint32_t e = (uint32_t)g;
            if (a.mode == 1) e = 2u * g + 18u * (uint32_t)abs((int)f[p] - (int)f[p - HW]);
            s1 += e;
            s2 += (uint64_t)e * e;
            const uint64_t n = (uint64_t)(t - a.t0 + 1);
            v = isqrt_u64(n * s2 - (uint64_t)s1 * s1);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((tid & 63) == 0) atomicAdd(&part[t - a.tb], v);
    }
    if (valid) {
        a.s1[p] = s1;
        a.s2[p] = s2;
    }
    __syncthreads();
    if (tid < a.te - a.tb) atomicAdd(&a.sout[tid], part[tid]);
}

// ------------------------------------------------------------ job set-up

__global__ __launch_bounds__(256) void init_jobs_kernel(const Job *jobs)
{
    const Job &J = jobs[blockIdx.y];
    const int i = blockIdx.x;
    if (i >= J.H) return;
    for (int j = threadIdx.x; j < J.W; j += 256) {
        J.M0[(size_t)i * J.Wp + j] = (int16_t)j;
        J.bmask[(size_t)i * J.W + j] = 0;
    }
    if (i == 0 && threadIdx.x == 0) {
        J.log[0] = J.W;
        J.log[1] = 0;
        J.log[2] = 0;
        J.log[3] = 0;
        J.state[0] = J.W <= J.Wt ? 0 : -1;
    }
}

// --------------------------------------------------------- uniform energy
//
// U(i, j) = floor(sum over the buffer's frames of e(i, j) / T) on the carved
// grid.  Carved pixel (i, j) of every frame of the buffer is original pixel
// (i, M(i, j)); the nine neighbours of the Sobel stencil are taken on the
// carved grid (replicated at the carved borders) and looked up through M.
// The difference term compares a frame with its carved predecessor, which
// for the buffer's first frame is frame t0 - 1 read through the same map.

__global__ __launch_bounds__(256) void energy_kernel(const Job *jobs, int r)
{
    const Job &J = jobs[blockIdx.z];
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    const int j = blockIdx.x * 64 + threadIdx.x;
    const int i = blockIdx.y * 4 + threadIdx.y;
    if (i >= J.H || j >= Wr) return;
    const int16_t *__restrict__ M = (r & 1) ? J.M1 : J.M0;
    const int Wp = J.Wp, W = J.W, H = J.H;
    const int im = max(i - 1, 0), ip = min(i + 1, H - 1), jm = max(j - 1, 0), jp = min(j + 1, Wr - 1);
    const int16_t *ma = M + (size_t)im * Wp, *mb = M + (size_t)i * Wp, *mc = M + (size_t)ip * Wp;
    const int oa0 = im * W + mcol(ma, jm, W), oa1 = im * W + mcol(ma, j, W), oa2 = im * W + mcol(ma, jp, W);
    const int ob0 = i * W + mcol(mb, jm, W), ob1 = i * W + mcol(mb, j, W), ob2 = i * W + mcol(mb, jp, W);
    const int oc0 = ip * W + mcol(mc, jm, W), oc1 = ip * W + mcol(mc, j, W), oc2 = ip * W + mcol(mc, jp, W);
    const size_t HW = (size_t)H * W;
    const uint8_t *f = J.luma + (size_t)J.t0 * HW;
    int acc = 0;
    if (J.mode == 1) {
        int prev = J.has_prev ? (int)f[(ptrdiff_t)ob1 - (ptrdiff_t)HW] : 0;
        for (int t = 0; t < J.T; ++t, f += HW) {
            const int c = f[ob1];
            const int g = sobel9(f[oa0], f[oa1], f[oa2], f[ob0], f[ob2], f[oc0], f[oc1], f[oc2]);
            const int d = (t > 0 || J.has_prev) ? abs(c - prev) : 0;
            acc += 2 * g + 18 * d;
            prev = c;
        }
    } else {
        for (int t = 0; t < J.T; ++t, f += HW)
            acc += sobel9(f[oa0], f[oa1], f[oa2], f[ob0], f[ob2], f[oc0], f[oc1], f[oc2]);
    }
    J.U[(size_t)i * Wp + j] = (uint16_t)(acc / J.T);
}

// ------------------------------------------------------------------- DP
//
// Eq. (4) row by row inside one workgroup of 1024 threads; thread t owns the
// Q consecutive columns [tQ, tQ + Q).  Each row needs the previous row's
// values of the two columns beside a thread's range, exchanged through a
// ping-pong pair of LDS slots so one barrier per row suffices.  Every pixel
// takes the leftmost of its least predecessors, its parent label (row-0
// column) and its indicator (predecessor column - column).

template <int Q>
__device__ __forceinline__ void store_dir(int8_t *p, const int (&d)[Q])
{
    if constexpr (Q == 1) {
        p[0] = (int8_t)d[0];
    } else if constexpr (Q == 2) {
        *reinterpret_cast<uint16_t *>(p) = (uint16_t)((d[0] & 255) | ((d[1] & 255) << 8));
    } else {
#pragma unroll
        for (int w = 0; w < Q / 4; ++w) {
            uint32_t v = (uint32_t)(d[4 * w] & 255) | ((uint32_t)(d[4 * w + 1] & 255) << 8) |
                         ((uint32_t)(d[4 * w + 2] & 255) << 16) | ((uint32_t)(d[4 * w + 3] & 255) << 24);
            reinterpret_cast<uint32_t *>(p)[w] = v;
        }
    }
}

template <int Q>
__global__ __launch_bounds__(kDpThreads) void dp_kernel(const Job *jobs, int r)
{
    const Job &J = jobs[blockIdx.x];
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    __shared__ int xce[2][2][kDpThreads];
    __shared__ int xlab[2][2][kDpThreads];
    const int tid = threadIdx.x;
    const int j0 = tid * Q;
    const int H = J.H, Wp = J.Wp;
    const uint16_t *__restrict__ U = J.U;
    int8_t *__restrict__ dir = J.dir;
    const bool owns = j0 < Wp;

    int ce[Q], lab[Q], un[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const int j = j0 + c;
        ce[c] = j < Wr ? (int)U[j] : kInf;
        lab[c] = j;
    }
    if (owns) {
        int z[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) z[c] = 0;
        store_dir<Q>(dir + j0, z);
    }
    xce[0][0][tid] = ce[0];
    xce[0][1][tid] = ce[Q - 1];
    xlab[0][0][tid] = lab[0];
    xlab[0][1][tid] = lab[Q - 1];
    if (H > 1) {
#pragma unroll
        for (int c = 0; c < Q; ++c) un[c] = (j0 + c) < Wr ? (int)U[(size_t)Wp + j0 + c] : 0;
    }
    __syncthreads();

    for (int i = 1; i < H; ++i) {
        const int p = (i - 1) & 1;
        int uc[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) uc[c] = un[c];
        if (i + 1 < H) {
            const uint16_t *row = U + (size_t)(i + 1) * Wp;
#pragma unroll
            for (int c = 0; c < Q; ++c) un[c] = (j0 + c) < Wr ? (int)row[j0 + c] : 0;
        }
        const int lce = tid > 0 ? xce[p][1][tid - 1] : kInf;
        const int llab = tid > 0 ? xlab[p][1][tid - 1] : 0;
        const int rce = tid < kDpThreads - 1 ? xce[p][0][tid + 1] : kInf;
        const int rlab = tid < kDpThreads - 1 ? xlab[p][0][tid + 1] : 0;
        int nce[Q], nlab[Q], d[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const int Lv = c == 0 ? lce : ce[c - 1];
            const int Ll = c == 0 ? llab : lab[c - 1];
            const int Rv = c == Q - 1 ? rce : ce[c + 1];
            const int Rl = c == Q - 1 ? rlab : lab[c + 1];
            int best = Lv, bl = Ll, dd = -1;
            if (ce[c] < best) {
                best = ce[c];
                bl = lab[c];
                dd = 0;
            }
            if (Rv < best) {
                best = Rv;
                bl = Rl;
                dd = 1;
            }
            const bool valid = (j0 + c) < Wr;
            nce[c] = valid ? uc[c] + best : kInf;
            nlab[c] = bl;
            d[c] = valid ? dd : 0;
        }
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            ce[c] = nce[c];
            lab[c] = nlab[c];
        }
        if (owns) store_dir<Q>(dir + (size_t)i * Wp + j0, d);
        const int q = i & 1;
        xce[q][0][tid] = ce[0];
        xce[q][1][tid] = ce[Q - 1];
        xlab[q][0][tid] = lab[0];
        xlab[q][1][tid] = lab[Q - 1];
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const int j = j0 + c;
        if (j < Wr) {
            J.ce_last[j] = ce[c];
            J.lab_last[j] = lab[c];
        }
    }
}

// ----------------------------------------------------------- band origins
//
// For band b (rows [lo, hi]) and every column j at row hi: follow the
// indicators up to row lo and, for b > 0, one more step into row lo - 1 (the
// last row of band b - 1).  borg[b][j] = reached column - j, |.| <= kBand.
// The band's indicator rows around the block's columns are staged in LDS.

__global__ __launch_bounds__(256) void borg_kernel(const Job *jobs, int r)
{
    const Job &J = jobs[blockIdx.z];
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    const int b = blockIdx.y;
    if (b >= J.nb) return;
    const int c0 = blockIdx.x * 256;
    if (c0 >= Wr) return;
    const int lo = b * kBand, hi = min(lo + kBand, J.H) - 1;
    const int rlo = max(lo, 1);
    const int nrows = hi - rlo + 1;  // 0 when the job has a single row
    const int wlo = max(c0 - nrows, 0), whi = min(c0 + 256 + nrows, Wr);
    const int ww = whi - wlo;
    __shared__ int8_t tile[kBand][256 + 2 * kBand];
    for (int idx = threadIdx.x; idx < nrows * ww; idx += 256) {
        const int rr = idx / ww, cc = idx - rr * ww;
        tile[rr][cc] = J.dir[(size_t)(rlo + rr) * J.Wp + wlo + cc];
    }
    __syncthreads();
    const int j = c0 + threadIdx.x;
    if (j < Wr) {
        int c = j;
        for (int i = hi; i >= rlo; --i) c += tile[i - rlo][c - wlo];
        J.borg[(size_t)b * J.Wp + j] = (int8_t)(c - j);
    }
}

// -------------------------------------------------------------- selection
//
// One workgroup per job.  (A) least child of every parent: atomicMin of the
// key (CE << 15 | column) at the parent's label -- the key order is the
// ranking order (CE, column) and the leftmost least child has the least key.
// (B) compact the parents' keys in label order, which is column order
// because labels never decrease along the row.  (C) k_iter = min(k, P_eff,
// W_r - Wt); a candidate is taken when fewer than k_iter keys are smaller.
// (D) the taken children in column order.  (E) every taken child walks the
// band origins upward to get its column at the last row of every band.

__device__ void band_jumps(const Job &J, int kk, const int8_t *bo, int bo_pitch, int tid, int nthreads)
{
    const int nb = J.nb;
    for (int s = tid; s < kk; s += nthreads) {
        int c = J.children[s];
        for (int b = nb - 1; b >= 0; --b) {
            J.bcol[s * nb + b] = c;
            if (b > 0) c += bo[(size_t)b * bo_pitch + c];
        }
    }
}

__global__ __launch_bounds__(1024) void select_kernel(const Job *jobs, int r, int lds_bytes)
{
    extern __shared__ uint64_t dsm[];
    __shared__ int scan_tmp[16];
    const Job &J = jobs[blockIdx.x];
    const int Wr = job_width(J, r);
    const int tid = threadIdx.x;
    if (Wr <= J.Wt) {
        if (tid == 0 && r + 1 < J.logcap) {
            J.log[4 * (r + 1)] = Wr;
            J.log[4 * (r + 1) + 1] = 0;
            J.log[4 * (r + 1) + 2] = 0;
        }
        return;
    }
    const bool in_lds = (size_t)2 * Wr * sizeof(uint64_t) <= (size_t)lds_bytes;
    uint64_t *key = in_lds ? dsm : J.keys;
    uint64_t *cand = key + Wr;
    constexpr uint64_t kNone = ~0ull;

    for (int j = tid; j < Wr; j += 1024) key[j] = kNone;
    __syncthreads();
    for (int j = tid; j < Wr; j += 1024) {
        const uint64_t kv = ((uint64_t)(uint32_t)J.ce_last[j] << 15) | (uint64_t)j;
        const int l = J.lab_last[j];
        if ((unsigned)l < (unsigned)Wr) atomicMin((unsigned long long *)&key[l], (unsigned long long)kv);
    }
    __syncthreads();

    const int chunk = (Wr + 1023) / 1024;
    const int l0 = min(tid * chunk, Wr), l1 = min(l0 + chunk, Wr);
    int cnt = 0;
    for (int l = l0; l < l1; ++l) cnt += key[l] != kNone;
    int peff = 0;
    int off = block_exclusive_scan(cnt, scan_tmp, &peff);
    for (int l = l0; l < l1; ++l)
        if (key[l] != kNone) cand[off++] = key[l];
    __syncthreads();

    const int kk = min(min(J.k, peff), Wr - J.Wt);
    const int chunk2 = (peff + 1023) / 1024;  // <= 32
    const int a0 = min(tid * chunk2, peff), a1 = min(a0 + chunk2, peff);
    uint32_t selmask = 0;
    int nsel = 0;
    for (int a = a0; a < a1; ++a) {
        const uint64_t x = cand[a];
        int rank = 0;
        for (int b = 0; b < peff && rank < kk; ++b) rank += cand[b] < x;
        if (rank < kk) {
            selmask |= 1u << (a - a0);
            ++nsel;
        }
    }
    int total = 0;
    int soff = block_exclusive_scan(nsel, scan_tmp, &total);
    for (int a = a0; a < a1; ++a)
        if (selmask & (1u << (a - a0))) J.children[soff++] = (int)(cand[a] & 0x7fff);
    __syncthreads();

    // band origins into LDS when they fit (the key arrays are dead by now)
    const int nb = J.nb;
    const bool bo_lds = (size_t)nb * Wr <= (size_t)lds_bytes;
    const int8_t *bo = J.borg;
    int bo_pitch = J.Wp;
    if (bo_lds && nb > 1) {
        int8_t *s = reinterpret_cast<int8_t *>(dsm);
        for (int idx = tid; idx < nb * Wr; idx += 1024) {
            const int b = idx / Wr, c = idx - b * Wr;
            s[idx] = J.borg[(size_t)b * J.Wp + c];
        }
        bo = s;
        bo_pitch = Wr;
        __syncthreads();
    }
    band_jumps(J, kk, bo, bo_pitch, tid, 1024);

    if (tid == 0) {
        J.log[4 * r + 1] = peff;
        J.log[4 * r + 2] = kk;
        if (r + 1 < J.logcap) {
            J.log[4 * (r + 1)] = Wr - kk;
            J.log[4 * (r + 1) + 1] = 0;
            J.log[4 * (r + 1) + 2] = 0;
            J.log[4 * (r + 1) + 3] = 0;
        }
        if (Wr - kk <= J.Wt) J.state[0] = r + 1;
    }
}

// Band jumps alone, for the backtrack stage entry point (children and
// k_iter already in place).
__global__ __launch_bounds__(256) void jump_kernel(const Job *jobs, int r)
{
    const Job &J = jobs[blockIdx.x];
    band_jumps(J, J.log[4 * r + 2], J.borg, J.Wp, threadIdx.x, 256);
}

// ------------------------------------------------------------------- fill
//
// One wavefront per (seam, band): the band's indicator rows in the window
// the seam can reach from its known bottom column are staged in LDS, one
// lane follows them upward, then the wave writes the seam's columns and
// marks the removed pixels (original columns, via the column map) in the
// buffer mask with the iteration number + 1.

__global__ __launch_bounds__(64) void fill_kernel(const Job *jobs, int r)
{
    const Job &J = jobs[blockIdx.z];
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    const int kk = J.log[4 * r + 2];
    const int b = blockIdx.y;
    if (b >= J.nb) return;
    const int H = J.H, nb = J.nb, lane = threadIdx.x;
    const int16_t *__restrict__ M = (r & 1) ? J.M1 : J.M0;
    __shared__ int8_t tile[kBand][2 * kBand];
    __shared__ int16_t path[kBand];
    const int lo = b * kBand, hi = min(lo + kBand, H) - 1;
    const int span = hi - lo;
    for (int s = blockIdx.x; s < kk; s += gridDim.x) {
        const int c_end = J.bcol[s * nb + b];
        const int wlo = max(c_end - span, 0), whi = min(c_end + span + 1, Wr);
        const int ww = whi - wlo;
        for (int idx = lane; idx < span * ww; idx += 64) {
            const int rr = idx / ww, cc = idx - rr * ww;
            tile[rr][cc] = J.dir[(size_t)(lo + 1 + rr) * J.Wp + wlo + cc];
        }
        __syncthreads();
        if (lane == 0) {
            int c = c_end;
            path[span] = (int16_t)c;
            for (int i = hi; i > lo; --i) {
                c += tile[i - lo - 1][c - wlo];
                path[i - 1 - lo] = (int16_t)c;
            }
        }
        __syncthreads();
        for (int rr = lane; rr <= span; rr += 64) {
            const int i = lo + rr;
            const int x = path[rr];
            J.seams[(size_t)s * H + i] = (int16_t)x;
            J.bmask[(size_t)i * J.W + mcol(M + (size_t)i * J.Wp, x, J.W)] = (uint16_t)(r + 1);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- compact
//
// Row i loses the k_iter columns R_0 < ... < R_{k-1} (seams never share a
// pixel and keep their order).  Output column j reads source column
// j + #{s : R_s - s <= j}; R_s - s never decreases, so a binary search
// finds the count.  Only the column map is compacted: frames stay put.

__global__ __launch_bounds__(256) void compact_kernel(const Job *jobs, int r)
{
    const Job &J = jobs[blockIdx.y];
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    const int i = blockIdx.x;
    if (i >= J.H) return;
    const int kk = J.log[4 * r + 2];
    const int H = J.H;
    const int16_t *__restrict__ Mc = ((r & 1) ? J.M1 : J.M0) + (size_t)i * J.Wp;
    int16_t *__restrict__ Mn = ((r & 1) ? J.M0 : J.M1) + (size_t)i * J.Wp;
    __shared__ int R[256];
    const bool lds = kk <= 256;
    if (lds) {
        for (int s = threadIdx.x; s < kk; s += 256) R[s] = J.seams[(size_t)s * H + i] - s;
        __syncthreads();
    }
    for (int j = threadIdx.x; j < Wr - kk; j += 256) {
        int a = 0, b = kk;
        while (a < b) {
            const int m = (a + b) >> 1;
            const int v = lds ? R[m] : (J.seams[(size_t)m * H + i] - m);
            if (v <= j) a = m + 1;
            else b = m;
        }
        Mn[j] = Mc[j + a];
    }
}

// ----------------------------------------------------------------- gather
//
// Carved output of every frame of the buffer: out(t, i, j) = frame(t, i,
// M(i, j)) for j < Wt, all channels; masks of every frame = buffer mask.

__global__ __launch_bounds__(256) void gather_kernel(const Job *jobs)
{
    const Job &J = jobs[blockIdx.y];
    const int i = blockIdx.x;
    if (i >= J.H) return;
    const int rd = J.state[0];
    const int16_t *__restrict__ M = ((rd & 1) ? J.M1 : J.M0) + (size_t)i * J.Wp;
    const int C = J.C, W = J.W, Wt = J.Wt, H = J.H;
    for (int t = J.t0; t < J.t0 + J.T; ++t) {
        const uint8_t *src = J.frames + ((size_t)t * H + i) * W * C;
        uint8_t *dst = J.out + ((size_t)t * H + i) * Wt * C;
        if (C == 1) {
            for (int j = threadIdx.x; j < Wt; j += 256) dst[j] = src[mcol(M, j, W)];
        } else {
            for (int idx = threadIdx.x; idx < Wt * C; idx += 256) {
                const int j = idx / C, c = idx - j * C;
                dst[idx] = src[mcol(M, j, W) * C + c];
            }
        }
        if (J.masks) {
            uint16_t *mdst = J.masks + ((size_t)t * H + i) * W;
            const uint16_t *msrc = J.bmask + (size_t)i * W;
            for (int j = threadIdx.x; j < W; j += 256) mdst[j] = msrc[j];
        }
    }
}

// ------------------------------------------------- stage-API conversions

__global__ void u32_to_u16_kernel(const int32_t *src, uint16_t *dst, int H, int W, int pitch)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p - (int64_t)i * W);
    dst[(size_t)i * pitch + j] = (uint16_t)src[p];
}

__global__ void u16_to_i32_kernel(const uint16_t *src, int32_t *dst, int H, int W, int pitch)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p - (int64_t)i * W);
    dst[p] = (int32_t)src[(size_t)i * pitch + j];
}

__global__ void i16_to_i32_kernel(const int16_t *src, int32_t *dst, int64_t n)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) dst[p] = src[p];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------- launchers

void launch_luma(const uint8_t *rgb, uint8_t *y, int64_t npx, hipStream_t s)
{
    if (npx <= 0) return;
    if ((((uintptr_t)rgb) | ((uintptr_t)y)) & 15)
        hipLaunchKernelGGL(luma_scalar_kernel, dim3(blocks_for(npx, 256)), dim3(256), 0, s, rgb, y, npx);
    else
        hipLaunchKernelGGL(luma_vec_kernel, dim3(blocks_for(npx, 256 * 16)), dim3(256), 0, s, rgb, y, npx);
}

void launch_seg_window(const SegArgs &a, hipStream_t s)
{
    const int64_t HW = (int64_t)a.H * a.W;
    hipLaunchKernelGGL(seg_window_kernel, dim3(blocks_for(HW, 256)), dim3(256), 0, s, a);
}

void launch_init_jobs(const Job *d_jobs, int njobs, int Hmax, int, hipStream_t s)
{
    hipLaunchKernelGGL(init_jobs_kernel, dim3(Hmax, njobs), dim3(256), 0, s, d_jobs);
}

void launch_energy(const Job *d_jobs, int njobs, int r, int Hmax, int Wmax, hipStream_t s)
{
    hipLaunchKernelGGL(energy_kernel, dim3(blocks_for(Wmax, 64), blocks_for(Hmax, 4), njobs), dim3(64, 4), 0, s,
                       d_jobs, r);
}

void launch_dp(const Job *d_jobs, int njobs, int r, int Wmax, hipStream_t s)
{
    const dim3 g(njobs), b(kDpThreads);
    if (Wmax <= 1024) hipLaunchKernelGGL(dp_kernel<1>, g, b, 0, s, d_jobs, r);
    else if (Wmax <= 2048) hipLaunchKernelGGL(dp_kernel<2>, g, b, 0, s, d_jobs, r);
    else if (Wmax <= 4096) hipLaunchKernelGGL(dp_kernel<4>, g, b, 0, s, d_jobs, r);
    else if (Wmax <= 8192) hipLaunchKernelGGL(dp_kernel<8>, g, b, 0, s, d_jobs, r);
    else if (Wmax <= 16384) hipLaunchKernelGGL(dp_kernel<16>, g, b, 0, s, d_jobs, r);
    else hipLaunchKernelGGL(dp_kernel<32>, g, b, 0, s, d_jobs, r);
}

void launch_borg(const Job *d_jobs, int njobs, int r, int nbmax, int Wmax, hipStream_t s)
{
    hipLaunchKernelGGL(borg_kernel, dim3(blocks_for(Wmax, 256), nbmax, njobs), dim3(256), 0, s, d_jobs, r);
}

void launch_select(const Job *d_jobs, int njobs, int r, int, int, size_t lds_cap, hipStream_t s)
{
    hipLaunchKernelGGL(select_kernel, dim3(njobs), dim3(1024), lds_cap, s, d_jobs, r, (int)lds_cap);
}

void launch_jump_only(const Job *d_jobs, int njobs, int r, hipStream_t s)
{
    hipLaunchKernelGGL(jump_kernel, dim3(njobs), dim3(256), 0, s, d_jobs, r);
}

void launch_fill(const Job *d_jobs, int njobs, int r, int kmax, int nbmax, hipStream_t s)
{
    const int gx = kmax < 1024 ? kmax : 1024;
    hipLaunchKernelGGL(fill_kernel, dim3(gx, nbmax, njobs), dim3(64), 0, s, d_jobs, r);
}

void launch_compact(const Job *d_jobs, int njobs, int r, int Hmax, hipStream_t s)
{
    hipLaunchKernelGGL(compact_kernel, dim3(Hmax, njobs), dim3(256), 0, s, d_jobs, r);
}

void launch_gather(const Job *d_jobs, int njobs, int Hmax, hipStream_t s)
{
    hipLaunchKernelGGL(gather_kernel, dim3(Hmax, njobs), dim3(256), 0, s, d_jobs);
}

void launch_u32_to_u16(const int32_t *src, uint16_t *dst, int H, int W, int pitch, hipStream_t s)
{
    hipLaunchKernelGGL(u32_to_u16_kernel, dim3(blocks_for((int64_t)H * W, 256)), dim3(256), 0, s, src, dst, H, W,
                       pitch);
}

void launch_u16_to_i32(const uint16_t *src, int32_t *dst, int H, int W, int pitch, hipStream_t s)
{
    hipLaunchKernelGGL(u16_to_i32_kernel, dim3(blocks_for((int64_t)H * W, 256)), dim3(256), 0, s, src, dst, H, W,
                       pitch);
}

void launch_i16_to_i32(const int16_t *src, int32_t *dst, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(i16_to_i32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, dst, n);
}

}  // namespace scpl
