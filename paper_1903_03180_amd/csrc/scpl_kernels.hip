// HIP kernels of libscpl.so for gfx950 (MI355X): SCPL video retargeting.
//
// Method: "Fast Video Retargeting Based on Seam Carving with Parental
// Labeling" (arXiv 1903.03180).  Stage map:
//   luma / tile_luma   colour -> 8-bit luma (the paper does not say which
//                      channel feeds the energy; BT.601 luma is used), tiled
//   seg_window_kernel  energy (Sec. 3.3) + ASDE moments (eqs. 7-8) for a
//                      window of candidate frames of one buffer (Sec. 3.2)
//   energy_kernel      uniform energy of a buffer (Sec. 3.2): mean of the
//                      frames' motion-aware energies, as 16-bit DP keys
//   dp_band_kernel     cumulative energy, eq. (4), one workgroup per buffer,
//                      leftmost tie-break, 2-bit indicator codes
//   borg_kernel        band origins of the two-level backtrack
//   select_kernel      row-0 parent labels through the band origins, per-
//                      parent least child (eq. 6), top-k, band jumps
//   fill_kernel        seams inside each band; buffer mask
//   update_kernel      removes the iteration's seams from the column map
//                      and the DP keys in one pass
//   refresh_kernel     recomputes the keys of the pixels whose carved 3x3
//                      neighbourhood changed (exact); ends the iteration
//   gather_kernel      carved output frames and masks
#include "scpl_internal.h"

namespace scpl {

namespace {

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack2(u16x2 v) { return (uint32_t)v.x | ((uint32_t)v.y << 16); }

__device__ __forceinline__ int job_width(const Job &J, int r) { return r < J.logcap ? J.log[4 * r] : J.Wt; }

// The job's current iteration: every kernel of an iteration reads it from
// the job's state, and the iteration's last kernel (the refresh) moves it on
// when its last workgroup for the job is done, so that each job advances at
// its own pace and a fixed sequence of launches (a graph) can be replayed for
// any number of iterations.
__device__ __forceinline__ int job_iter(const Job &J) { return J.state[3]; }

// Global-address-space views of pointers held in job descriptors.  Loads
// through generic pointers compile to flat instructions, which also count
// against the LDS wait counter, so every wait for an LDS access would drain
// the outstanding global loads too (and defeat prefetching).
#define GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLOBAL T *gp(T *p)
{
    return (GLOBAL T *)p;
}
template <class T>
__device__ __forceinline__ const GLOBAL T *gp(const T *p)
{
    return (const GLOBAL T *)p;
}

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

// floor(sqrt(q)).  Below 2^40 (the common case): q as a float (two
// conversions and one fma, relative error below 2^-23), the hardware single
// precision square root (within 1 ulp), so the estimate of a root below 2^20
// is off by less than 0.35 and its integer part by at most 1, which one
// integer comparison either way repairs.  Otherwise: the hardware
// reciprocal square root in double precision, one Newton step (relative
// error then far below 2^-40, so the estimate is within 1 of the root for
// every q < 2^64), then integer steps until exact.
__device__ __forceinline__ uint32_t isqrt_u64(uint64_t q)
{
    if (q < (1ull << 40)) {
        const float qf = fmaf((float)(uint32_t)(q >> 32), 4294967296.0f, (float)(uint32_t)q);
        uint32_t r = (uint32_t)__builtin_amdgcn_sqrtf(qf);
        const uint64_t r2 = (uint64_t)r * r;
        if (r2 > q) --r;
        else if (r2 + 2 * (uint64_t)r + 1 <= q) ++r;
        return r;
    }
    const double qd = (double)(uint32_t)(q >> 32) * 4294967296.0 + (double)(uint32_t)q;
    double y = __builtin_amdgcn_rsq(qd);
    y = y * (1.5 - 0.5 * qd * y * y);
    uint64_t r = (uint64_t)(uint32_t)min(qd * y, 4294967295.0);
    while (r * r > q) --r;
    while (r < 0xffffffffull && (r + 1) * (r + 1) <= q) ++r;
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

// Tiled luma: a block converts a strip of 16 rows x 128 columns of one
// frame (row-major, C channels) into 16 consecutive tiles.  The strip is
// read row by row (coalesced), converted into LDS, and written as 2 KB of
// contiguous tiles.  Columns past W are zero (never read).
__global__ __launch_bounds__(256) void tile_luma_kernel(const uint8_t *__restrict__ src, int C, int N, int H, int W,
                                                        uint8_t *__restrict__ dst, int vec)
{
    __shared__ uint8_t strip[16][128];
    const int ntc = tiles_across(W);
    const int c0 = blockIdx.y * 128;            // first column of the strip
    const int r0 = (blockIdx.x % ((H + 15) / 16)) * 16;
    const int n = blockIdx.x / ((H + 15) / 16);
    const int tid = threadIdx.x;
    // 16 rows x 128 columns: thread -> (row tid / 16, 8 columns from (tid % 16) * 8)
    const int rr = tid >> 4, cc = (tid & 15) * 8;
    const int r = r0 + rr, c = c0 + cc;
    uint32_t lo = 0, hi = 0;
    if (r < H && c < W) {
        const uint8_t *row = src + ((size_t)n * H + r) * (size_t)W * C;
        if (vec && c + 8 <= W) {
            if (C == 3) {
                const u32x2 *q = reinterpret_cast<const u32x2 *>(row + (size_t)c * 3);
                const u32x2 a = q[0], b = q[1], d = q[2];
                const uint32_t w[6] = {a.x, a.y, b.x, b.y, d.x, d.y};
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int k0 = 3 * k, k1 = 3 * k + 1, k2 = 3 * k + 2;
                    const uint32_t R = (w[k0 >> 2] >> (8 * (k0 & 3))) & 255u;
                    const uint32_t G = (w[k1 >> 2] >> (8 * (k1 & 3))) & 255u;
                    const uint32_t B = (w[k2 >> 2] >> (8 * (k2 & 3))) & 255u;
                    const uint32_t v = (77u * R + 150u * G + 29u * B + 128u) >> 8;
                    if (k < 4) lo |= v << (8 * k);
                    else hi |= v << (8 * (k - 4));
                }
            } else {
                const u32x2 a = *reinterpret_cast<const u32x2 *>(row + c);
                lo = a.x;
                hi = a.y;
            }
        } else {
            for (int k = 0; k < 8 && c + k < W; ++k) {
                const uint8_t *p = row + (size_t)(c + k) * C;
                const uint32_t v = C == 3 ? (77u * p[0] + 150u * p[1] + 29u * p[2] + 128u) >> 8 : p[0];
                if (k < 4) lo |= v << (8 * k);
                else hi |= v << (8 * (k - 4));
            }
        }
    }
    *reinterpret_cast<uint32_t *>(&strip[rr][cc]) = lo;
    *reinterpret_cast<uint32_t *>(&strip[rr][cc + 4]) = hi;
    __syncthreads();
    // 16 tiles of 16 rows x 8 columns: thread -> (tile tid / 16, tile row tid % 16)
    const int tile = tid >> 4, trow = tid & 15;
    const int tc = (c0 >> 3) + tile;
    if (tc < ntc && r0 + trow < H) {
        u32x2 o;
        o.x = *reinterpret_cast<const uint32_t *>(&strip[trow][tile * 8]);
        o.y = *reinterpret_cast<const uint32_t *>(&strip[trow][tile * 8 + 4]);
        *reinterpret_cast<u32x2 *>(dst + (size_t)n * tiled_frame_bytes(H, W) + tofs(r0 + trow, tc * 8, ntc)) = o;
    }
}

__global__ __launch_bounds__(256) void untile_kernel(const uint8_t *__restrict__ src, int N, int H, int W,
                                                     uint8_t *__restrict__ dst)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)N * H * W) return;
    const int c = (int)(p % W);
    const int64_t nr = p / W;
    const int r = (int)(nr % H), n = (int)(nr / H);
    dst[p] = src[(size_t)n * tiled_frame_bytes(H, W) + tofs(r, c, tiles_across(W))];
}

// ---------------------------------------------- tile-row energy helpers
//
// A thread works on one tile row: 8 consecutive columns of one row of a
// tiled luma frame.  row10 loads the 8 bytes with one 64-bit load plus the
// column on each side (replicated at the frame borders, as are rows above
// and below the frame); sobel8 then gives |Gx| + |Gy| of the 8 pixels from
// three such rows.  Columns of the last tile past the frame's width are
// filled with the last column, so every pixel's stencil is the replicated
// one.

// b[k] = luma of column 8 tc + k - 1 of row r (clamped into the frame).
__device__ __forceinline__ void row10(const GLOBAL uint8_t *f, int r, int H, int tc, int ntc, int W, int (&b)[10])
{
    r = min(max(r, 0), H - 1);
    const GLOBAL uint8_t *t = f + ((size_t)((r >> 4) * ntc + tc) << 7) + ((r & 15) << 3);
    const u32x2 v = *reinterpret_cast<const GLOBAL u32x2 *>(t);
    const int nv = W - 8 * tc;  // columns of this tile inside the frame (>= 1)
    // neighbours in the tiles left and right (same row); clamped addresses so
    // that every lane loads
    const int left = t[tc > 0 ? -121 : 0];
    const int right = t[nv > 8 ? 128 : 0];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        b[1 + k] = (int)((v.x >> (8 * k)) & 255u);
        b[5 + k] = (int)((v.y >> (8 * k)) & 255u);
    }
    b[0] = tc > 0 ? left : b[1];
    b[9] = right;
#pragma unroll
    for (int k = 2; k <= 9; ++k)
        if (k - 1 >= nv) b[k] = b[k - 1];  // past the last column: replicate it
}

// |Gx| + |Gy| of the 8 pixels of row b (rows a above, c below).
__device__ __forceinline__ void sobel8(const int (&a)[10], const int (&b)[10], const int (&c)[10], int (&g)[8])
{
    int v[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) v[k] = a[k] + 2 * b[k] + c[k];
#pragma unroll
    for (int x = 0; x < 8; ++x) {
        const int gx = v[x + 2] - v[x];
        const int gy = (c[x] + 2 * c[x + 1] + c[x + 2]) - (a[x] + 2 * a[x + 1] + a[x + 2]);
        g[x] = abs(gx) + abs(gy);
    }
}

// 8 bytes of row r (clamped) of a tiled frame at tile column tc.
__device__ __forceinline__ u32x2 row8(const GLOBAL uint8_t *f, int r, int H, int tc, int ntc)
{
    r = min(max(r, 0), H - 1);
    return *reinterpret_cast<const GLOBAL u32x2 *>(f + ((size_t)((r >> 4) * ntc + tc) << 7) + ((r & 15) << 3));
}

__device__ __forceinline__ int byte_of(const u32x2 &v, int x) { return (int)(((x < 4 ? v.x : v.y) >> (8 * (x & 3))) & 255u); }

// Energies of the 8 pixels of row r of frame f (Sec. 3.3); pf is the
// predecessor frame or null.  a, b, c: rows r - 1, r, r + 1 from row10.
__device__ __forceinline__ void energy8(const int (&a)[10], const int (&b)[10], const int (&c)[10],
                                        const GLOBAL uint8_t *pf, int r, int H, int tc, int ntc, int mode,
                                        uint32_t (&e)[8])
{
    int g[8];
    sobel8(a, b, c, g);
    if (mode != 1) {
#pragma unroll
        for (int x = 0; x < 8; ++x) e[x] = (uint32_t)g[x];
        return;
    }
    u32x2 p{0u, 0u};
    if (pf) p = row8(pf, r, H, tc, ntc);
#pragma unroll
    for (int x = 0; x < 8; ++x) e[x] = (uint32_t)(2 * g[x] + (pf ? 18 * abs(b[x + 1] - byte_of(p, x)) : 0));
}

// ------------------------------------------------------ pixel-major luma
//
// The refresh reads the same few pixels in every frame of a buffer; a
// pixel-major copy of the clip's luma makes those reads 16 frames wide.
// Entries s = 16 c + u of pixel p (p = row W + column) are at
// seq[(c H W + p) 16 + u]: 16 entries of a pixel are one 16-byte piece and
// the pieces of neighbouring pixels are neighbours.  Entry 0 is a copy of
// frame 0, entry s > 0 frame s - 1, entries past N copies of frame N - 1
// (seqp, the entries per pixel, is a multiple of 16 above N).  A block of
// 128 threads takes one tile of 16 rows x 8 columns: per 16 entries it loads
// the 16 frames' tiles with 16-byte loads into LDS, then each thread writes
// its pixel's piece with one 16-byte store.

__global__ __launch_bounds__(128) void seq_kernel(const uint8_t *__restrict__ tiled, int N, int H, int W, int64_t FS,
                                                  int ntc, uint8_t *__restrict__ seq, int seqp)
{
    __shared__ __align__(16) uint8_t buf[16 * 128];  // 16 entries x one tile
    const int tile = blockIdx.x;                    // tile row x ntc + tile column
    const int tr = tile / ntc, tc = tile - tr * ntc;
    const int tid = threadIdx.x;
    // the pixel of byte tid of the tile: row tid / 8, column tid % 8 of the tile
    const int r = tr * kTileH + (tid >> 3), j = tc * kTileW + (tid & 7);
    const bool live = r < H && j < W;
    const size_t HW = (size_t)H * W;
    GLOBAL uint8_t *dst = gp(seq) + ((size_t)r * W + j) * 16;
    for (int c = 0; c < seqp / 16; ++c) {
        // thread tid loads bytes [16 (tid % 8), +16) of the tile of entry 16 c + tid / 8
        const int f = min(max(16 * c + (tid >> 3) - 1, 0), N - 1);
        const u32x4 v = *reinterpret_cast<const GLOBAL u32x4 *>(gp(tiled) + (size_t)f * FS + (size_t)tile * 128 +
                                                                16 * (tid & 7));
        __syncthreads();  // the previous chunk's reads of buf are done
        *reinterpret_cast<u32x4 *>(buf + 16 * tid) = v;
        __syncthreads();
        if (live) {
            uint32_t w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                w[k] = (uint32_t)buf[(4 * k) * 128 + tid] | ((uint32_t)buf[(4 * k + 1) * 128 + tid] << 8) |
                       ((uint32_t)buf[(4 * k + 2) * 128 + tid] << 16) | ((uint32_t)buf[(4 * k + 3) * 128 + tid] << 24);
            *reinterpret_cast<GLOBAL u32x4 *>(dst + (size_t)c * HW * 16) = u32x4{w[0], w[1], w[2], w[3]};
        }
    }
}

// ------------------------------------------------------- ASDE window scan
//
// A thread holds 8 columns x 2 rows of the original frame (one tile row in
// each of two consecutive rows).  For a buffer starting at t0 whose moments
// S1 = sum e, S2 = sum e^2 cover frames [t0, tb), frames [tb, te) are
// appended one at a time; after each one the per-pixel
// floor(sqrt(n S2 - S1^2)) (n times the population deviation of eq. 8) is
// summed into sout[t - tb].  The host then decides every candidate in order
// (eq. 9) and discards the tail after the first rejection.

constexpr int kSegRows = 2;

// Energies of the kSegRows x 8 pixels from row r0, tile column tc, of tiled
// frame t (with the difference to frame t - 1 when diff).
__device__ __forceinline__ void seg_energies(const uint8_t *luma, int64_t FS, int t, bool diff, int r0, int H, int tc,
                                             int ntc, int W, int mode, uint32_t (&e)[kSegRows][8])
{
    const GLOBAL uint8_t *f = gp(luma) + (size_t)t * FS;
    const GLOBAL uint8_t *pf = diff ? f - FS : nullptr;
    int ra[10], rb[10], rc[10];
    row10(f, r0 - 1, H, tc, ntc, W, ra);
    row10(f, r0, H, tc, ntc, W, rb);
#pragma unroll
    for (int q = 0; q < kSegRows; ++q) {
        row10(f, r0 + q + 1, H, tc, ntc, W, rc);
        energy8(ra, rb, rc, pf, r0 + q, H, tc, ntc, mode, e[q]);
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            ra[k] = rb[k];
            rb[k] = rc[k];
        }
    }
}

__global__ __launch_bounds__(256) void seg_window_kernel(const SegArgs *args)
{
    __shared__ unsigned long long part[kSegWindow];
    const SegArgs &a = args[blockIdx.z];  // one clip's window per grid layer
    if ((int)blockIdx.x * 64 >= a.ntc || (int)blockIdx.y * 4 * kSegRows >= a.H) return;
    const int tid = threadIdx.x;
    if (tid < kSegWindow) part[tid] = 0;
    __syncthreads();
    const int n = a.ntc;
    const int tc = blockIdx.x * 64 + (tid >> 2);
    const int r0 = (blockIdx.y * 4 + (tid & 3)) * kSegRows;
    const bool valid = tc < n && r0 < a.H;
    const int tcc = valid ? tc : 0;
    const int nv = min(a.W - 8 * tcc, 8);
    const int64_t FS = a.FS;
    uint32_t s1[kSegRows][8];
    uint64_t s2[kSegRows][8];
    auto energies = [&](int t, bool diff, uint32_t (&e)[kSegRows][8]) {
        seg_energies(a.luma, FS, t, diff, r0, a.H, tcc, n, a.W, a.mode, e);
    };
    if (valid) {
        if (a.init) {
            uint32_t e[kSegRows][8];
            energies(a.t0, a.mode == 1 && a.t0 > 0, e);
#pragma unroll
            for (int q = 0; q < kSegRows; ++q)
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    s1[q][x] = e[q][x];
                    s2[q][x] = (uint64_t)e[q][x] * e[q][x];
                }
        } else {
#pragma unroll
            for (int q = 0; q < kSegRows; ++q)
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    const int i = min(r0 + q, a.H - 1), j = 8 * tcc + min(x, nv - 1);
                    s1[q][x] = a.s1[(int64_t)i * a.W + j];
                    s2[q][x] = a.s2[(int64_t)i * a.W + j];
                }
        }
    }
    for (int t = a.tb; t < a.te; ++t) {
        unsigned long long v = 0;
        if (valid) {
            uint32_t e[kSegRows][8];
            energies(t, a.mode == 1, e);
            const uint64_t nn = (uint64_t)(t - a.t0 + 1);
#pragma unroll
            for (int q = 0; q < kSegRows; ++q)
#pragma unroll
                for (int x = 0; x < 8; ++x) {
                    s1[q][x] += e[q][x];
                    s2[q][x] += (uint64_t)e[q][x] * e[q][x];
                    const bool in = r0 + q < a.H && x < nv;
                    v += in ? isqrt_u64(nn * s2[q][x] - (uint64_t)s1[q][x] * s1[q][x]) : 0u;
                }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if ((tid & 63) == 0) atomicAdd(&part[t - a.tb], v);
    }
    if (valid) {
#pragma unroll
        for (int q = 0; q < kSegRows; ++q)
#pragma unroll
            for (int x = 0; x < 8; ++x)
                if (r0 + q < a.H && x < nv) {
                    const int64_t p = (int64_t)(r0 + q) * a.W + 8 * tcc + x;
                    a.s1[p] = s1[q][x];
                    a.s2[p] = s2[q][x];
                }
    }
    __syncthreads();
    if (tid < a.te - a.tb) atomicAdd(&a.sout[tid], part[tid]);
}

// A finished buffer [t0, t0 + T) whose moments the window scans left
// covering frames [t0, thi): S1 less the energies of the frames [tlo, thi)
// scanned past its end (tlo = t0 + T) is the sum over its frames of the
// energy maps, and 4 floor(S1 / T) its first DP key rows (Sec. 3.2, the
// uniform energy of the buffer), written to out (H x W).  The energies are
// those of the window scan, so the difference is exact.
__global__ __launch_bounds__(256) void seg_finish_kernel(const SegFinish *args)
{
    const SegFinish &a = args[blockIdx.z];
    const int tid = threadIdx.x;
    const int tc = blockIdx.x * 64 + (tid >> 2);
    const int r0 = (blockIdx.y * 4 + (tid & 3)) * kSegRows;
    if (tc >= a.ntc || r0 >= a.H) return;
    const int nv = min(a.W - 8 * tc, 8);
    uint32_t acc[kSegRows][8];
#pragma unroll
    for (int q = 0; q < kSegRows; ++q)
#pragma unroll
        for (int x = 0; x < 8; ++x)
            acc[q][x] = (r0 + q < a.H && x < nv) ? a.s1[(int64_t)(r0 + q) * a.W + 8 * tc + x] : 0u;
    for (int t = a.tlo; t < a.thi; ++t) {
        uint32_t e[kSegRows][8];
        seg_energies(a.luma, a.FS, t, a.mode == 1, r0, a.H, tc, a.ntc, a.W, a.mode, e);
#pragma unroll
        for (int q = 0; q < kSegRows; ++q)
#pragma unroll
            for (int x = 0; x < 8; ++x) acc[q][x] -= e[q][x];
    }
    const uint32_t T = (uint32_t)a.T;
#pragma unroll
    for (int q = 0; q < kSegRows; ++q)
#pragma unroll
        for (int x = 0; x < 8; ++x)
            if (r0 + q < a.H && x < nv) a.out[(int64_t)(r0 + q) * a.W + 8 * tc + x] = (uint16_t)((acc[q][x] / T) << 2);
}

// ------------------------------------------------------------ job set-up

// Keys in registers: all ones is "no path".  Key rows in memory hold 16 bits
// per column, 0xffff beyond the width: 65535 per row exceeds what any real
// column can add in a row (4 x 7650 + 2, U <= 16382 in general), so by
// induction over the rows such a column's cumulative key always exceeds its
// real neighbour's and it never becomes anyone's predecessor.
constexpr uint32_t kKeyInf = 0xffffffffu;
constexpr uint16_t kRowInf = 0xffffu;

__global__ __launch_bounds__(256) void init_jobs_kernel(const Job *jobs)
{
    const Job &J = jobs[blockIdx.y];
    const int i = blockIdx.x;
    if (i > J.H) return;
    if (i == J.H) {  // the all-ones row read by DP lanes past the job's width
        for (int j = threadIdx.x; j < J.Kp; j += 256) {
            J.K[(size_t)i * J.Kp + j] = kRowInf;
        }
        return;
    }
    for (int j = threadIdx.x; j < J.W; j += 256) {
        J.M[(size_t)i * J.Wp + j] = (int16_t)j;
        J.bmask[(size_t)i * J.W + j] = 0;
    }
    for (int x = threadIdx.x; x < J.Kp; x += 256) {
        if (x >= J.KL && x < J.KL + J.W) continue;
        J.K[(size_t)i * J.Kp + x] = kRowInf;
    }
    if (i == 0 && threadIdx.x == 0) {
        J.log[0] = J.W;
        J.log[1] = 0;
        J.log[2] = 0;
        J.log[3] = 0;
        J.state[0] = J.W <= J.Wt ? 0 : -1;
        J.state[1] = J.W;
        J.state[2] = 0;
        J.state[3] = 0;
    }
}

// ------------------------------------------------------------ energy
//
// e of frame t at carved pixel (i, j), Sec. 3.3: the Sobel stencil is taken
// on the carved grid (rows i-1..i+1, columns j-1..j+1, replicated at the
// carved borders) and every carved pixel is read as original pixel
// (row, M(row, column)).  The difference term compares the frame with its
// carved predecessor: frame t-1, or for the buffer's first frame the frame
// just before the buffer (read through the same map), or nothing for the
// clip's first frame.

struct Stencil {
    int pa0, pa1, pa2, pb0, pb1, pb2, pc0, pc1, pc2;  // pixels (original row W + original column)
};

// Stencil of carved pixel (i, j) from the column-map rows of i-1, i, i+1
// (ma, mb, mc: carved column -> original column).
__device__ __forceinline__ Stencil stencil_from_rows(const int16_t *ma, const int16_t *mb, const int16_t *mc, int im,
                                                     int i, int ip, int j, int Wcur, int W)
{
    const int jm = max(j - 1, 0), jp = min(j + 1, Wcur - 1);
    Stencil s;
    s.pa0 = im * W + mcol(ma, jm, W);
    s.pa1 = im * W + mcol(ma, j, W);
    s.pa2 = im * W + mcol(ma, jp, W);
    s.pb0 = i * W + mcol(mb, jm, W);
    s.pb1 = i * W + mcol(mb, j, W);
    s.pb2 = i * W + mcol(mb, jp, W);
    s.pc0 = ip * W + mcol(mc, jm, W);
    s.pc1 = ip * W + mcol(mc, j, W);
    s.pc2 = ip * W + mcol(mc, jp, W);
    return s;
}

// Sum over the buffer's frames of the energy at a stencil (Sec. 3.3), from
// the clip's pixel-major luma (seq_kernel): entry 0 of a pixel is a copy of
// frame 0 and entry s > 0 frame s - 1.  Buffer frame t
// (clip frame t0 + t) is entry t0 + 1 + t and its predecessor entry t0 + t,
// which for the clip's first frame is frame 0 itself (no difference term).
// Entries come 16 at a time: ten 16-byte loads (the nine stencil pixels and
// the centre's previous 16) serve 16 frames.  Chunks c1, c1 + step, ... of
// the entries [t0 + 1, t0 + T] are summed; c1 and step are the same in
// every lane.
__device__ __forceinline__ uint32_t seq_sum(const Job &J, const Stencil &st, int c1, int step)
{
    const GLOBAL uint8_t *q = gp(J.seq);
    const size_t piece = (size_t)J.H * J.W * 16;  // bytes per chunk of 16 entries
    const bool motion = J.mode == 1;
    const int s_lo = J.t0 + 1, s_hi = J.t0 + J.T;  // entries of the buffer's frames
    const int cfirst = s_lo >> 4, clast = s_hi >> 4;
    const int pix[10] = {st.pa0, st.pa1, st.pa2, st.pb0, st.pb2, st.pc0, st.pc1, st.pc2, st.pb1, st.pb1};
    uint32_t acc = 0;
    for (int c = cfirst + c1; c <= clast; c += step) {
        u32x4 v[10];
#pragma unroll
        for (int k = 0; k < 9; ++k)
            v[k] = *reinterpret_cast<const GLOBAL u32x4 *>(q + (size_t)c * piece + 16 * (size_t)pix[k]);
        // the centre's 16 entries before this chunk (the predecessor of the first)
        v[9] = *reinterpret_cast<const GLOBAL u32x4 *>(q + (size_t)max(c - 1, 0) * piece + 16 * (size_t)pix[9]);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = 16 * c + u;
            auto byte = [&](const u32x4 &w, int x) { return (int)((w[x >> 2] >> (8 * (x & 3))) & 255u); };
            const int g = sobel9(byte(v[0], u), byte(v[1], u), byte(v[2], u), byte(v[3], u), byte(v[4], u),
                                 byte(v[5], u), byte(v[6], u), byte(v[7], u));
            const int prev = u > 0 ? byte(v[8], u - 1) : byte(v[9], 15);
            const uint32_t en = motion ? (uint32_t)(2 * g + 18 * abs(byte(v[8], u) - prev)) : (uint32_t)g;
            acc += (e >= s_lo && e <= s_hi) ? en : 0u;
        }
    }
    return acc;
}

// Iteration 0 of every job: the DP key row 4 floor(sum of the T energy
// maps / T) over the uncarved frames (the column map is the identity).  A
// thread sums 8 columns x 4 rows (one tile row in each of 4 consecutive
// rows) over the buffer's frames; a block covers 512 columns x 16 rows.
__global__ __launch_bounds__(256) void energy_kernel(const Job *jobs)
{
    const Job &J = jobs[blockIdx.z];
    if (J.W <= J.Wt) return;
    const int tid = threadIdx.x;
    const int n = J.ntc, H = J.H, W = J.W;
    const int tc = blockIdx.x * 64 + (tid >> 2);
    const int r0 = blockIdx.y * 16 + (tid & 3) * 4;
    if (tc >= n || r0 >= H) return;
    const int nv = min(W - 8 * tc, 8);
    if (J.u0) {  // the key rows the segmentation left (seg_finish_kernel)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = r0 + q;
            if (i >= H) break;
            const uint16_t *src = J.u0 + (size_t)i * W + 8 * tc;
            uint16_t *dst = J.K + (size_t)i * J.Kp + J.KL + 8 * tc;
#pragma unroll
            for (int x = 0; x < 8; ++x)
                if (x < nv) dst[x] = src[x];
        }
        return;
    }
    uint32_t acc[4][8];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int x = 0; x < 8; ++x) acc[q][x] = 0;
    for (int t = 0; t < J.T; ++t) {
        const GLOBAL uint8_t *f = gp(J.luma) + (size_t)(J.t0 + t) * J.FS;
        const GLOBAL uint8_t *pf = (J.mode == 1 && (t > 0 || J.has_prev)) ? f - J.FS : nullptr;
        int ra[10], rb[10], rc[10];
        row10(f, r0 - 1, H, tc, n, W, ra);
        row10(f, r0, H, tc, n, W, rb);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            row10(f, r0 + q + 1, H, tc, n, W, rc);
            uint32_t e[8];
            energy8(ra, rb, rc, pf, r0 + q, H, tc, n, J.mode, e);
#pragma unroll
            for (int x = 0; x < 8; ++x) acc[q][x] += e[x];
#pragma unroll
            for (int k = 0; k < 10; ++k) {
                ra[k] = rb[k];
                rb[k] = rc[k];
            }
        }
    }
    const uint32_t T = (uint32_t)J.T;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = r0 + q;
        if (i >= H) break;
        uint32_t k8[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) k8[x] = (acc[q][x] / T) << 2;
        uint16_t *dst = J.K + (size_t)i * J.Kp + J.KL + 8 * tc;  // 16-byte aligned
        if (nv == 8) {
            *gp(reinterpret_cast<u32x4 *>(dst)) =
                u32x4{k8[0] | (k8[1] << 16), k8[2] | (k8[3] << 16), k8[4] | (k8[5] << 16), k8[6] | (k8[7] << 16)};
        } else {
#pragma unroll
            for (int x = 0; x < 8; ++x)
                if (x < nv) dst[x] = (uint16_t)k8[x];
        }
    }
}

// ------------------------------------------------------------------- DP
//
// Eq. (4) row by row inside one workgroup; thread t owns the Q consecutive
// columns [tQ, tQ + Q).  Each column keeps key = CE * 4.  The three
// candidates of a pixel get the offsets 0 (left), 1 (above), 2 (right), so
// one unsigned min3 picks the least cumulative energy and, among equal
// ones, the leftmost; the offset left in the two low bits is the indicator
// code (predecessor column - column + 1).  Key rows hold 4 U in 16 bits and
// 0xffff at and beyond the current width (such columns never win, see
// kRowInf); values all ones in registers (no neighbour) stay all ones
// through saturating adds.  Neighbours inside a wavefront come through
// DPP wave shifts; the two wavefront-edge values cross through LDS, one
// barrier per row.  Key rows are requested a group of PF rows ahead.
// Parent labels are not carried here: they follow from the band origins.

__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) { return __builtin_elementwise_add_sat(a, b); }

// A pointer that is the same in every lane, moved into scalar registers
// (buffer resources built from it then need no per-lane loop).
template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T *>(((uint64_t)hi << 32) | lo);
}

// Q consecutive 16-bit keys of one row, as loaded (two per word).
template <int Q>
struct KRow {
    uint32_t w[(Q + 1) / 2];
    __device__ __forceinline__ uint32_t at(int c) const
    {
        if constexpr (Q == 1) return w[0];
        return (c & 1) ? (w[c >> 1] >> 16) : (w[c >> 1] & 0xffffu);
    }
};

template <int Q>
__device__ __forceinline__ void load_krow(KRow<Q> &dst, const uint16_t *p)
{
    if constexpr (Q == 1) {
        dst.w[0] = *gp(p);
    } else if constexpr (Q == 2) {
        dst.w[0] = *gp(reinterpret_cast<const uint32_t *>(p));
    } else if constexpr (Q == 4) {
        const u32x2 v = *gp(reinterpret_cast<const u32x2 *>(p));
        dst.w[0] = v.x;
        dst.w[1] = v.y;
    } else {
#pragma unroll
        for (int q = 0; q < Q / 8; ++q) {
            const u32x4 v = gp(reinterpret_cast<const u32x4 *>(p))[q];
            dst.w[4 * q] = v.x;
            dst.w[4 * q + 1] = v.y;
            dst.w[4 * q + 2] = v.z;
            dst.w[4 * q + 3] = v.w;
        }
    }
}

// The same through a buffer resource: byte offset voff (per lane) plus soff
// (wave-uniform, a scalar operand of the load, so a row step needs no
// 64-bit address arithmetic).
template <int Q>
__device__ __forceinline__ void load_krow_buf(KRow<Q> &dst, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    static_assert(Q == 2 || Q == 4 || Q % 8 == 0, "whole 32-, 64- or 128-bit loads");
    if constexpr (Q == 2) {
        dst.w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
    } else if constexpr (Q == 4) {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
        dst.w[0] = v.x;
        dst.w[1] = v.y;
    } else {
#pragma unroll
        for (int q = 0; q < Q / 8; ++q) {
            const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(voff + 16u * q), (int)soff, 0);
            dst.w[4 * q] = v.x;
            dst.w[4 * q + 1] = v.y;
            dst.w[4 * q + 2] = v.z;
            dst.w[4 * q + 3] = v.w;
        }
    }
}

// Stores the low byte of each best key; readers keep its two low bits.
template <int Q>
__device__ __forceinline__ void store_codes(uint8_t *p, const uint32_t (&b)[Q])
{
    if constexpr (Q == 1) {
        gp(p)[0] = (uint8_t)b[0];
    } else if constexpr (Q == 2) {
        *gp(reinterpret_cast<uint16_t *>(p)) = (uint16_t)__builtin_amdgcn_perm(b[1], b[0], 0x0c0c0400u);
    } else {
#pragma unroll
        for (int w = 0; w < Q / 4; ++w) {
            const uint32_t lo = __builtin_amdgcn_perm(b[4 * w + 1], b[4 * w], 0x0c0c0400u);
            const uint32_t hi = __builtin_amdgcn_perm(b[4 * w + 3], b[4 * w + 2], 0x0c0c0400u);
            gp(reinterpret_cast<uint32_t *>(p))[w] = lo | (hi << 16);
        }
    }
}

template <int Q>
struct DpPrefetch {
    static constexpr int PF = Q <= 4 ? 8 : (Q == 8 ? 4 : 2);  // row-synchronous kernel
};

// One DP row step of a lane holding Q consecutive columns: lnb / rnb are the
// previous row's keys just left / right of the lane; nxt the key row.
template <int Q>
__device__ __forceinline__ void dp_step(uint32_t (&key)[Q], uint32_t lnb, uint32_t rnb, const KRow<Q> &nxt,
                                        uint32_t (&best)[Q])
{
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const uint32_t kl = c == 0 ? lnb : key[c - 1];
        const uint32_t kc = sat_add(key[c], 1u);
        const uint32_t kr = sat_add(c == Q - 1 ? rnb : key[c + 1], 2u);
        best[c] = min(min(kl, kc), kr);
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) key[c] = sat_add(nxt.at(c), best[c] & ~3u);
}

// Row-synchronous DP for the widest frames: every row, the two
// wavefront-edge keys cross through LDS and the block meets at a barrier.
template <int Q>
__global__ __launch_bounds__(1024) void dp_kernel(const Job *jobs)
{
    constexpr int PF = DpPrefetch<Q>::PF;
    const Job &J = jobs[blockIdx.x];
    const int r = job_iter(J);
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    __shared__ uint32_t eL[2][16], eR[2][16];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int nwave = blockDim.x >> 6;
    const int j0 = tid * Q;
    const int H = J.H, Kp = J.Kp, Wp = J.Wp;
    const bool owns = J.KL + j0 + Q <= Kp;
    const uint16_t *K = J.K;
    // lanes past the job's key rows read the all-ones row at stride 0
    const uint16_t *kp = owns ? K + J.KL + j0 : K + (size_t)H * Kp;
    const size_t kstride = owns ? (size_t)Kp : 0;
    uint8_t *__restrict__ dir = J.dir;
    const bool stores = j0 < Wp;

    uint32_t key[Q];
    {
        KRow<Q> k0;
        load_krow<Q>(k0, kp);
        uint32_t code[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            key[c] = k0.at(c);
            code[c] = 1;
        }
        if (stores) store_codes<Q>(dir + j0, code);
    }
    if (lane == 0) eL[0][wid] = key[0];
    if (lane == 63) eR[0][wid] = key[Q - 1];

    KRow<Q> cur[PF], nxt[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s) load_krow<Q>(cur[s], kp + (size_t)min(1 + s, H - 1) * kstride);
    __syncthreads();

    for (int i0 = 1; i0 < H; i0 += PF) {
#pragma unroll
        for (int s = 0; s < PF; ++s) load_krow<Q>(nxt[s], kp + (size_t)min(i0 + PF + s, H - 1) * kstride);
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            const int i = i0 + s;
            if (i < H) {
                const int p = (i - 1) & 1;
                uint32_t lnb = (uint32_t)__builtin_amdgcn_update_dpp((int)kKeyInf, (int)key[Q - 1], 0x138, 0xf, 0xf,
                                                                     false);
                uint32_t rnb = (uint32_t)__builtin_amdgcn_update_dpp((int)kKeyInf, (int)key[0], 0x130, 0xf, 0xf,
                                                                     false);
                if (lane == 0) lnb = wid > 0 ? eR[p][wid - 1] : kKeyInf;
                if (lane == 63) rnb = wid < nwave - 1 ? eL[p][wid + 1] : kKeyInf;
                uint32_t best[Q];
                dp_step<Q>(key, lnb, rnb, cur[s], best);
                if (stores) store_codes<Q>(dir + (size_t)i * Wp + j0, best);
                const int q = i & 1;
                if (lane == 0) eL[q][wid] = key[0];
                if (lane == 63) eR[q][wid] = key[Q - 1];
                __syncthreads();
            }
        }
#pragma unroll
        for (int s = 0; s < PF; ++s) cur[s] = nxt[s];
    }
#pragma unroll
    for (int c = 0; c < Q; ++c) {
        const int j = j0 + c;
        if (j < Wr) J.ce_last[j] = (int)(key[c] >> 2);
    }
}

// Banded DP.  Wavefront w owns the C = 64 Q - 2 HB columns [wC, wC + C) and
// also computes HB columns on each side of them: its lanes cover columns
// [wC - HB, wC + C + HB), neighbours within the wavefront come through DPP
// wave shifts and the two outermost neighbours count as all ones.  Starting
// from a row that is exact over the whole cover, the error from the
// outermost neighbours advances one column per row, so after HB rows the
// owned columns are still exact.  At the end of each band of HB rows the
// owners publish their keys of the band's last row in LDS (ping-pong), the
// block meets at one barrier, and the halo lanes take the neighbours' keys.
// Only owned columns keep indicator codes.
//
// Key rows are read PF rows at a time into two register sets used in turn
// (no copies between them), so a group of rows is requested a whole group
// ahead of its use and waiting for it never waits for the codes stored
// since.  Row addresses are wave-uniform (scalar) plus a fixed 32-bit byte
// offset per lane.  Variants with a deep key prefetch (Q PF >= 64) are
// limited to 512 threads, which doubles the registers a lane may use.
__host__ __device__ constexpr int dp_max_threads(int Q, int PF) { return Q * PF >= 64 ? 512 : 1024; }

template <int Q>
__device__ __forceinline__ void load_krow_at(KRow<Q> &dst, const char *row, uint32_t off)
{
    load_krow<Q>(dst, reinterpret_cast<const uint16_t *>(row + off));
}

// Whether row s of a group of PF rows (groups start at rows 1 + n PF) can
// open a band of HB rows (bands start at rows 1 + m HB).
__host__ __device__ constexpr bool dp_band_row(int s, int HB, int PF)
{
    return PF % HB == 0 ? s % HB == 0 : (HB % PF == 0 ? s == 0 : true);
}

// Rows [i1, i_end) in groups of PF rows, from two register sets of key rows
// used in turn.  The first group runs before the loop, so that every entry
// into the loop has the same memory operations in flight (one group of key
// loads, then one group of code stores).  With the first group inside the
// loop, its entry from above has no stores in flight, and the compiler's
// wait for each key row, which must hold on both entries, then also waits
// on the back edge for a code store of the previous group (gfx9's vmcnt
// counts stores too).
template <int PF, class KR, class Fetch, class Group>
__device__ __forceinline__ void dp_rows(KR (&ka)[PF], KR (&kb)[PF], int i1, int i_end, Fetch &&fetch, Group &&group)
{
    fetch(ka, i1);
    fetch(kb, i1 + PF);
    if (i1 + PF > i_end) {
        group(ka, i1, true);
        return;
    }
    group(ka, i1, false);
    int i0 = i1 + PF;
    for (; i0 + 2 * PF <= i_end; i0 += 2 * PF) {
        fetch(ka, i0 + PF);
        group(kb, i0, false);
        fetch(kb, i0 + 2 * PF);
        group(ka, i0 + PF, false);
    }
    if (i0 < i_end) {
        fetch(ka, i0 + PF);
        group(kb, i0, true);
        if (i0 + PF < i_end) group(ka, i0 + PF, true);
    }
}

template <int Q, int HB, int PF>
__global__ __launch_bounds__(dp_max_threads(Q, PF)) void dp_band_kernel(const Job *jobs)
{
    constexpr int C = 64 * Q - 2 * HB;
    static_assert(HB % Q == 0 && C > 0, "halo must be whole lanes");
    extern __shared__ uint32_t rowbuf[];  // 2 x (Kp - KL) keys
    const Job &J = jobs[blockIdx.x];
    const int r = job_iter(J);
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int H = J.H, Kp = J.Kp, Wp = J.Wp;
    const int rb = Kp - J.KL;  // keys per row buffer
    const int jl = wid * C - HB + lane * Q;  // first column of this lane (>= -KL)
    const bool live = wid < J.dpnw;          // wave-uniform
    const bool owner = live && lane * Q >= HB && lane * Q < HB + C;
    const bool stores = owner && jl < Wp;
    // waves past the job's columns read the all-ones row, at stride 0
    const uint16_t *K = J.K;
    const char *kbase = reinterpret_cast<const char *>(live ? K : K + (size_t)H * Kp);
    const uint32_t kpitch = live ? (uint32_t)Kp * 2u : 0u;  // key rows span < 4 GiB
    const uint32_t koff = live ? (uint32_t)(J.KL + jl) * 2u : 0u;
    const uint32_t rlast = (uint32_t)(H - 1) * kpitch;
    const __amdgpu_buffer_rsrc_t krs =
        __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(kbase), (short)0, 0x7fffffff, 0x00020000);
    // every lane stores its codes each row: lanes whose codes are not kept
    // (halo, past the width) write to the job's scratch row instead, so
    // the row loop has no branch around the store
    uint8_t *__restrict__ dir = J.dir;
    uint32_t coff = stores ? (uint32_t)jl : (uint32_t)(H * Wp + lane * Q);
    const uint32_t cstep = stores ? (uint32_t)Wp : 0u;

    uint32_t key[Q];
    {
        KRow<Q> k0;
        load_krow_at<Q>(k0, kbase, koff);
        uint32_t code[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            key[c] = k0.at(c);
            code[c] = 1;
        }
        store_codes<Q>(dir + coff, code);
        coff += cstep;
    }
    // neighbour registers: lane 0's left and lane 63's right stay all ones
    uint32_t lnb = kKeyInf, rnb = kKeyInf;
    int band_left = HB;  // rows left in the current band
    int buf = 0;

    auto fetch = [&](KRow<Q>(&kr)[PF], int i0) {
        uint32_t ro = (uint32_t)i0 * kpitch;
#pragma unroll
        for (int s = 0; s < PF; ++s, ro += kpitch) load_krow_buf<Q>(kr[s], krs, koff, min(ro, rlast));
    };
    auto step = [&](const KRow<Q> &kr) {
        lnb = (uint32_t)__builtin_amdgcn_update_dpp((int)lnb, (int)key[Q - 1], 0x138, 0xf, 0xf, false);
        rnb = (uint32_t)__builtin_amdgcn_update_dpp((int)rnb, (int)key[0], 0x130, 0xf, 0xf, false);
        uint32_t best[Q];
        dp_step<Q>(key, lnb, rnb, kr, best);
        store_codes<Q>(dir + coff, best);
        coff += cstep;
        --band_left;
    };
    auto exchange = [&]() {
        // publish the band's last row, meet, refresh the halo
        uint32_t *rowp = rowbuf + (size_t)buf * rb;
        if (owner) {
#pragma unroll
            for (int c = 0; c < Q; ++c) rowp[jl + c] = key[c];
        }
        __syncthreads();
        if (live && !owner) {
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const int j = jl + c;
                key[c] = (j >= 0 && j < Wr) ? rowp[j] : kKeyInf;
            }
        }
        buf ^= 1;
        band_left = HB;
    };
    // rows i0 .. i0 + PF - 1 from kr; `guard` for the last, partial groups
    auto group = [&](const KRow<Q>(&kr)[PF], int i0, bool guard) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            if (guard && i0 + s >= H) break;
            if (dp_band_row(s, HB, PF)) {
                if (band_left == 0) exchange();
            }
            step(kr[s]);
        }
    };

    KRow<Q> ka[PF], kb[PF];
    dp_rows<PF>(ka, kb, 1, H, fetch, group);
    if (owner) {
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const int j = jl + c;
            if (j >= 0 && j < Wr) J.ce_last[j] = (int)(key[c] >> 2);
        }
    }
}

// Column-split DP over a chunk of R rows: several workgroups per buffer, one
// launch per chunk.  Workgroup g owns the columns [A, B) = [g P, (g + 1) P)
// (clipped to W_r) and covers [X0, X0 + nwv C) with X0 = max(A - R, 0): as
// in dp_band_kernel each wavefront owns C columns of the cover, computes HB
// more on each side and meets the others every HB rows through LDS.
// Columns outside the cover count as all ones, so the cover loses one exact
// column per row at each inner edge; after R rows the owned columns are
// still exact.  A chunk starts from the previous chunk's last row of 32-bit
// keys (two rows per buffer, used by consecutive chunks in turn; columns
// outside the frame start at all ones, which like the 0xffff padding never
// wins) and leaves its own last row there; the first chunk starts from key
// row 0, the last writes the last row's CE.  With fewer columns per lane
// than one workgroup per buffer can afford, a row costs fewer instructions
// per wavefront, and the launch boundaries replace any wait between
// workgroups.
// Workgroup gx of the chunk of rows [r0, r0 + R) of job J in iteration r
// (width Wr > Wt), with nthreads threads; rowbuf: 2 x nwv C keys of LDS.
template <int Q, int HB, int PF>
__device__ __forceinline__ void dp_chunk_body(const Job &J, int Wr, int gx, int r0, int R, int P, int nthreads,
                                              uint32_t *rowbuf)
{
    constexpr int C = 64 * Q - 2 * HB;
    static_assert(HB % Q == 0 && C > 0, "halo must be whole lanes");
    const int H = J.H, Kp = J.Kp, Wp = J.Wp;
    if (r0 >= H) return;
    const int A = gx * P;
    if (A >= Wr) return;
    const int B = min(A + P, Wr);
    const int Bs = B == Wr ? Wp : B;  // the last workgroup also stores the padding codes
    const int nwv = nthreads >> 6;
    const int cw = nwv * C;
    const int X0 = max(A - R, 0);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int jl = X0 + wid * C - HB + lane * Q;  // first column of this lane (>= -HB)
    const bool wown = lane * Q >= HB && lane * Q < HB + C;  // the wavefront's own columns
    const bool stores = wown && jl >= A && jl < Bs;
    const int ci = r0 / R;  // chunk index
    const int i_end = min(r0 + R, H);
    const char *kbase = reinterpret_cast<const char *>(J.K);
    const uint32_t kpitch = (uint32_t)Kp * 2u;
    const uint32_t koff = (uint32_t)(J.KL + jl) * 2u;
    const uint32_t rlast = (uint32_t)(H - 1) * kpitch;
    // the resource spans the key rows and the all-ones row after them
    const uint32_t nrec = (uint32_t)(H + 1) * kpitch;
    const __amdgpu_buffer_rsrc_t krs =
        __builtin_amdgcn_make_buffer_rsrc((void *)uniform_ptr(kbase), (short)0, (int)nrec, 0x00020000);
    uint8_t *__restrict__ dir = J.dir;
    uint32_t coff = stores ? (uint32_t)jl : (uint32_t)(H * Wp + lane * Q);
    const uint32_t cstep = stores ? (uint32_t)Wp : 0u;

    uint32_t key[Q];
    int i1;  // first row computed from the previous one
    if (r0 == 0) {
        KRow<Q> k0;
        load_krow_at<Q>(k0, kbase, koff);
        uint32_t code[Q];
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            key[c] = k0.at(c);
            code[c] = 1;
        }
        store_codes<Q>(dir + coff, code);
        i1 = 1;
    } else {
        const uint32_t *bk = J.bk + (size_t)((ci - 1) & 1) * Wp;
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const int j = jl + c;
            key[c] = (j >= 0 && j < Wr) ? bk[j] : kKeyInf;
        }
        i1 = r0;
    }
    coff += cstep * (uint32_t)i1;
    uint32_t lnb = kKeyInf, rnb = kKeyInf;
    int band_left = HB;
    int buf = 0;

    // Only the columns within T - t of the owned ones at step t of T can still
    // reach them, so a lane's key row is needed up to row i_end - 1 plus its
    // distance to [A, B) (negative outside).  Beyond that the lane reads past
    // the end of the buffer resource (offset nrec, out of range whether or not
    // the row offset is counted), which returns zeros and moves no data.
    const int lastrow = i_end - 1 + min(jl + Q - 1 - A, B - 1 - jl);
    auto fetch = [&](KRow<Q>(&kr)[PF], int i0) {
        // decided once per group, by its first row: a lane still needed there
        // reads the whole group
        const uint32_t vo = i0 <= lastrow ? koff : nrec;
        uint32_t ro = (uint32_t)i0 * kpitch;
#pragma unroll
        for (int s = 0; s < PF; ++s, ro += kpitch) load_krow_buf<Q>(kr[s], krs, vo, min(ro, rlast));
    };
    auto step = [&](const KRow<Q> &kr) {
        lnb = (uint32_t)__builtin_amdgcn_update_dpp((int)lnb, (int)key[Q - 1], 0x138, 0xf, 0xf, false);
        rnb = (uint32_t)__builtin_amdgcn_update_dpp((int)rnb, (int)key[0], 0x130, 0xf, 0xf, false);
        uint32_t best[Q];
        dp_step<Q>(key, lnb, rnb, kr, best);
        store_codes<Q>(dir + coff, best);
        coff += cstep;
        --band_left;
    };
    auto exchange = [&]() {
        uint32_t *rowp = rowbuf + (size_t)buf * cw;
        if (wown) {
#pragma unroll
            for (int c = 0; c < Q; ++c) rowp[jl + c - X0] = key[c];
        }
        __syncthreads();
        if (!wown) {
#pragma unroll
            for (int c = 0; c < Q; ++c) {
                const int j = jl + c;
                key[c] = (j >= X0 && j < X0 + cw && j < Wr) ? rowp[j - X0] : kKeyInf;
            }
        }
        buf ^= 1;
        band_left = HB;
    };
    auto group = [&](const KRow<Q>(&kr)[PF], int i0, bool guard) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            if (guard && i0 + s >= i_end) break;
            if (band_left == 0) exchange();
            step(kr[s]);
        }
    };

    KRow<Q> ka[PF], kb[PF];
    dp_rows<PF>(ka, kb, i1, i_end, fetch, group);
    // the chunk's last row: the next chunk's start, or the last row's CE
    const bool last = i_end == H;
    uint32_t *bko = J.bk + (size_t)(ci & 1) * Wp;
    if (wown) {
#pragma unroll
        for (int c = 0; c < Q; ++c) {
            const int j = jl + c;
            if (j >= A && j < B) {
                if (last) J.ce_last[j] = (int)(key[c] >> 2);
                else bko[j] = key[c];
            }
        }
    }
}

// Workgroups go to the eight XCDs in turn by their number, and each XCD has
// an L2 of its own.  The ngx workgroups of a job read overlapping covers
// (neighbours share 2R columns), so with xcd_local they are numbered to land
// on one XCD: workgroup gx of job y is number 8 (gx + ngx floor(y / 8)) +
// y mod 8, in a grid of ngx ceil(njobs / 8) 8 workgroups (those past the
// last job return); otherwise it is number gx + ngx y.
template <int Q, int HB, int PF>
__global__ __launch_bounds__(dp_max_threads(Q, PF)) void dp_chunk_kernel(const Job *jobs, int njobs, int ngx,
                                                                          int xcd_local, int r0, int R, int P)
{
    extern __shared__ uint32_t rowbuf[];  // 2 x nwv C keys: the cover
    const int L = (int)blockIdx.x;
    const int job = xcd_local ? 8 * ((L >> 3) / ngx) + (L & 7) : L / ngx;
    const int gx = xcd_local ? (L >> 3) % ngx : L % ngx;
    if (job >= njobs) return;
    const Job &J = jobs[job];
    const int r = __builtin_amdgcn_readfirstlane(job_iter(J));
    const int Wr = __builtin_amdgcn_readfirstlane(job_width(J, r));
    if (Wr <= J.Wt) return;
    dp_chunk_body<Q, HB, PF>(J, Wr, gx, r0, R, P, (int)blockDim.x, rowbuf);
}

// ----------------------------------------------------------- band origins
//
// For band b (rows [lo, hi]) and every column j at row hi: follow the
// indicators up to row lo and, for b > 0, one more step into row lo - 1 (the
// last row of band b - 1); for b = 0 up to row 0.  borg[b][j] = reached
// column - j, |.| <= B.  The band's indicator rows around the block's 128
// columns are staged in LDS with 32-bit loads.

constexpr int kBorgCols = 256;  // columns per workgroup of the default variant

__device__ __forceinline__ int code_step(uint8_t c) { return (int)(c & 3u) - 1; }

// Copies rows [r0, r0 + nrows) x columns [c0, c1) of a byte matrix with a
// pitch that is a multiple of 4 into LDS (pitch lp bytes, column c0 & ~3 at
// LDS column 0), using aligned 32-bit loads.  Each thread requests its next
// eight words before it writes any of them (words past the staged rows
// read 0 through the buffer resource and are not written).  src, pitch,
// r0, nrows, c0 and c1 are the same in every thread.  Returns the LDS
// column of c0.
__device__ __forceinline__ int stage_bytes(uint8_t *lds, int lp, const uint8_t *src, int pitch, int r0, int nrows,
                                           int c0, int c1, int tid, int nthreads)
{
    const int a0 = c0 & ~3;
    const int nw = (c1 - a0 + 3) >> 2;  // words per row
    if (nw <= 0 || nrows <= 0) return c0 - a0;
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)uniform_ptr(src), (short)0, __builtin_amdgcn_readfirstlane((r0 + nrows) * pitch), 0x00020000);
    // (row, word) of this thread, advanced by nthreads words per step
    int rr = tid / nw, w = tid - rr * nw;
    const int drr = nthreads / nw, dw = nthreads - drr * nw;
    constexpr int kBatch = 8;
    while (rr < nrows) {
        uint32_t v[kBatch];
        int at[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            at[u] = rr < nrows ? rr * lp + 4 * w : -1;
            v[u] = __builtin_amdgcn_raw_buffer_load_b32(rsrc, (r0 + rr) * pitch + a0 + 4 * w, 0, 0);
            rr += drr;
            w += dw;
            if (w >= nw) {
                w -= nw;
                ++rr;
            }
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (at[u] >= 0) *reinterpret_cast<uint32_t *>(lds + at[u]) = v[u];
    }
    return c0 - a0;
}

// Columns [c0, c0 + COLS) of band b of job J (width Wr); COLS threads;
// tile: B rows x (COLS + 2B + 8) bytes of LDS.
template <int COLS>
__device__ __forceinline__ void borg_body(const Job &J, int Wr, int b, int c0, uint8_t *tile)
{
    const int B = J.B;
    const int lo = b * B, hi = min(lo + B, J.H) - 1;
    const int rlo = max(lo, 1);
    const int nrows = hi - rlo + 1;  // 0 when the job has a single row
    const int wlo = max(c0 - nrows, 0), whi = min(c0 + COLS + nrows, Wr);
    const int lp = COLS + 2 * B + 8;
    const int sh = stage_bytes(tile, lp, J.dir, J.Wp, rlo, nrows, wlo, whi, threadIdx.x, COLS) - wlo;
    __syncthreads();
    const int j = c0 + threadIdx.x;
    if (j < Wr) {
        int c = j;
        for (int i = hi; i >= rlo; --i) c += code_step(tile[(i - rlo) * lp + c + sh]);
        J.borg[(size_t)b * J.Wp + j] = (int8_t)(c - j);
    }
}

template <int COLS>
__global__ __launch_bounds__(COLS) void borg_kernel(const Job *jobs)
{
    extern __shared__ uint8_t tile[];  // B rows x (COLS + 2B + 8) bytes
    const Job &J = jobs[blockIdx.z];
    const int r = job_iter(J);
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    const int b = blockIdx.y;
    if (b >= J.nb) return;
    const int c0 = blockIdx.x * COLS;
    if (c0 >= Wr) return;
    borg_body<COLS>(J, Wr, b, c0, tile);
}

// Parent labels of the last row from the band origins (stage entry point
// of the DP): label(j) = column reached at row 0 from (H-1, j).
__global__ __launch_bounds__(256) void labels_kernel(const Job *jobs)
{
    const Job &J = jobs[blockIdx.y];
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= J.W) return;
    int c = j;
    for (int b = J.nb - 1; b >= 0; --b) c += J.borg[(size_t)b * J.Wp + c];
    J.lab_last[j] = c;
}

// -------------------------------------------------------------- selection
//
// One workgroup per job.  (A) parent label of every last-row pixel (the
// row-0 column its seam reaches, Sec. 3.1), by following the band origins;
// least child of every parent: atomicMin of the key (CE << 15 | column) at
// the label -- the key order is the ranking order (CE, column) and the
// leftmost least child has the least key.  (B) compact the parents' keys in
// label order, which is column order because labels never decrease along
// the row.  (C) k_iter = min(k, P_eff, W_r - Wt); a candidate is taken when
// fewer than k_iter keys are smaller.  (D) the taken children in column
// order.  (E) every taken child walks the band origins upward to get its
// column at the last row of every band.

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

// Selection of job J in iteration r (width Wr > Wt) by NT threads; dsm:
// lds_bytes of LDS, scan_tmp: 16 ints of LDS.  NT = 256 serves widths up to
// 8192 (32 candidates per thread at most).
template <int NT>
__device__ __forceinline__ void select_body(const Job &J, int r, int Wr, int lds_bytes, int use_lab_array,
                                            uint64_t *dsm, int *scan_tmp)
{
    const int tid = threadIdx.x;
    const int nb = J.nb;
    const size_t key_bytes = (size_t)2 * Wr * sizeof(uint64_t);
    const bool keys_lds = key_bytes <= (size_t)lds_bytes;
    const size_t key_room = keys_lds ? key_bytes : 0;
    const int bo_lp = (Wr + 3 + 4) & ~3;  // staged rows may start up to 3 bytes early
    const bool bo_lds = (size_t)nb * bo_lp + key_room <= (size_t)lds_bytes;
    uint64_t *key = keys_lds ? dsm : J.keys;
    uint64_t *cand = key + Wr;
    uint8_t *bo_s = reinterpret_cast<uint8_t *>(dsm) + key_room;
    const int8_t *bo = bo_lds ? reinterpret_cast<const int8_t *>(bo_s) : J.borg;
    const int bo_pitch = bo_lds ? bo_lp : J.Wp;
    // band origins that do not all fit beside the keys: staged G bands at a
    // time, and the label and jump walks advance group by group (their
    // positions kept in the candidate half of the key array)
    const int G = !bo_lds ? (int)(((size_t)lds_bytes - key_room) / (size_t)bo_lp) : 0;
    const bool grouped = G >= 2 && !use_lab_array;
    constexpr uint64_t kNone = ~0ull;
    auto stage_bands = [&](int lo, int hi) {
        __syncthreads();  // the previous group's rows are read
        stage_bytes(bo_s, bo_lp, reinterpret_cast<const uint8_t *>(J.borg), J.Wp, lo, hi - lo + 1, 0, Wr, tid, NT);
        __syncthreads();
    };

    if (grouped) {
        int *lab = reinterpret_cast<int *>(cand);
        for (int j = tid; j < Wr; j += NT) {
            key[j] = kNone;
            lab[j] = j;
        }
        for (int hi = nb - 1; hi >= 0; hi -= G) {
            const int lo = max(hi - G + 1, 0);
            stage_bands(lo, hi);
            for (int j = tid; j < Wr; j += NT) {
                int l = lab[j];
                for (int b = hi; b >= lo; --b) l += (int8_t)bo_s[(b - lo) * bo_lp + l];
                lab[j] = l;
            }
        }
        __syncthreads();
        for (int j = tid; j < Wr; j += NT) {
            const int l = lab[j];
            const uint64_t kv = ((uint64_t)(uint32_t)J.ce_last[j] << 15) | (uint64_t)j;
            if ((unsigned)l < (unsigned)Wr) atomicMin((unsigned long long *)&key[l], (unsigned long long)kv);
        }
    } else {
        for (int j = tid; j < Wr; j += NT) key[j] = kNone;
        if (bo_lds) stage_bytes(bo_s, bo_lp, reinterpret_cast<const uint8_t *>(J.borg), J.Wp, 0, nb, 0, Wr, tid, NT);
        __syncthreads();
        for (int j = tid; j < Wr; j += NT) {
            int l;
            if (use_lab_array) {
                l = J.lab_last[j];
            } else {
                l = j;
                for (int b = nb - 1; b >= 0; --b) l += bo[(size_t)b * bo_pitch + l];
            }
            const uint64_t kv = ((uint64_t)(uint32_t)J.ce_last[j] << 15) | (uint64_t)j;
            if ((unsigned)l < (unsigned)Wr) atomicMin((unsigned long long *)&key[l], (unsigned long long)kv);
        }
    }
    __syncthreads();

    const int chunk = (Wr + NT - 1) / NT;
    const int l0 = min(tid * chunk, Wr), l1 = min(l0 + chunk, Wr);
    int cnt = 0;
    for (int l = l0; l < l1; ++l) cnt += key[l] != kNone;
    int peff = 0;
    int off = block_exclusive_scan(cnt, scan_tmp, &peff);
    for (int l = l0; l < l1; ++l)
        if (key[l] != kNone) cand[off++] = key[l];
    __syncthreads();

    const int kk = min(min(J.k, peff), Wr - J.Wt);
    const int chunk2 = (peff + NT - 1) / NT;  // <= 32
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

    if (grouped) {
        // every taken child walks the band origins upward, G bands at a time
        int *cpos = reinterpret_cast<int *>(cand);
        for (int q = tid; q < kk; q += NT) cpos[q] = J.children[q];
        for (int hi = nb - 1; hi >= 0; hi -= G) {
            const int lo = max(hi - G + 1, 0);
            stage_bands(lo, hi);
            for (int q = tid; q < kk; q += NT) {
                int c = cpos[q];
                for (int b = hi; b >= lo; --b) {
                    J.bcol[q * nb + b] = c;
                    if (b > 0) c += (int8_t)bo_s[(b - lo) * bo_lp + c];
                }
                cpos[q] = c;
            }
        }
    } else {
        band_jumps(J, kk, bo, bo_pitch, tid, NT);
    }

    if (tid == 0) {
        J.log[4 * r + 1] = peff;
        J.log[4 * r + 2] = kk;
        if (r + 1 < J.logcap) {
            J.log[4 * (r + 1)] = Wr - kk;
            J.log[4 * (r + 1) + 1] = 0;
            J.log[4 * (r + 1) + 2] = 0;
            J.log[4 * (r + 1) + 3] = 0;
        }
        J.state[1] = Wr - kk;
        J.state[2] = kk;
        if (Wr - kk <= J.Wt) J.state[0] = r + 1;
    }
}

__global__ __launch_bounds__(1024) void select_kernel(const Job *jobs, int lds_bytes, int use_lab_array)
{
    extern __shared__ uint64_t dsm[];
    __shared__ int scan_tmp[16];
    const Job &J = jobs[blockIdx.x];
    const int r = job_iter(J);
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) {
        if (threadIdx.x == 0 && r + 1 < J.logcap) {
            J.log[4 * (r + 1)] = Wr;
            J.log[4 * (r + 1) + 1] = 0;
            J.log[4 * (r + 1) + 2] = 0;
        }
        return;
    }
    select_body<1024>(J, r, Wr, lds_bytes, use_lab_array, dsm, scan_tmp);
}

// Band jumps alone, for the backtrack stage entry point (children and
// k_iter already in place).
__global__ __launch_bounds__(256) void jump_kernel(const Job *jobs)
{
    const Job &J = jobs[blockIdx.x];
    const int r = job_iter(J);
    band_jumps(J, J.log[4 * r + 2], J.borg, J.Wp, threadIdx.x, 256);
}

// ------------------------------------------------------------------- fill
//
// One wavefront per (seam, band): the band's indicator rows in the window
// the seam can reach from its known bottom column are staged in LDS, one
// lane follows them upward, then the wave writes the seam's columns and
// marks the removed pixels (original columns, via the column map) in the
// buffer mask with the iteration number + 1.

__global__ __launch_bounds__(64) void fill_kernel(const Job *jobs)
{
    extern __shared__ uint8_t tile[];  // B - 1 rows x (2 B + 8) bytes of the launch's largest B
    __shared__ int16_t path[kBandMax];
    const Job &J = jobs[blockIdx.z];
    const int r = job_iter(J);
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;
    const int kk = J.log[4 * r + 2];
    const int b = blockIdx.y;
    if (b >= J.nb) return;
    const int H = J.H, nb = J.nb, lane = threadIdx.x;
    const int fp = 2 * J.B + 8;  // LDS pitch: the window of a seam is at most 2 B - 1 wide, staged from a word
    const int16_t *__restrict__ M = J.M;
    const int lo = b * J.B, hi = min(lo + J.B, H) - 1;
    const int span = hi - lo;  // < B <= kBandMax
    for (int s = blockIdx.x; s < kk; s += gridDim.x) {
        const int c_end = J.bcol[s * nb + b];
        const int wlo = max(c_end - span, 0), whi = min(c_end + span + 1, Wr);
        const int sh = stage_bytes(tile, fp, J.dir, J.Wp, lo + 1, span, wlo, whi, lane, 64) - wlo;
        __syncthreads();
        if (lane == 0) {
            int c = c_end;
            path[span] = (int16_t)c;
            for (int i = hi; i > lo; --i) {
                c += code_step(tile[(i - lo - 1) * fp + c + sh]);
                path[i - 1 - lo] = (int16_t)c;
            }
        }
        __syncthreads();
        for (int rr = lane; rr <= span; rr += 64) {
            const int i = lo + rr;
            const int x = path[rr];
            J.seams[(size_t)i * J.kcap + s] = (int16_t)x;
            J.bmask[(size_t)i * J.W + mcol(M + (size_t)i * J.Wp, x, J.W)] = (uint16_t)(r + 1);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ compact + update
//
// Row i loses the k_iter columns R_0 < ... < R_{k-1} (seams never share a
// pixel and keep their order).  New column j of a row reads old column
// j + #{s : R_s - s <= j}; R_s - s never decreases, so a binary search
// finds the count.  Only the column map is compacted: frames stay put.
//
// The DP key row 4 floor(SE / T) (SE = sum of the buffer's energy maps) is
// carried the same way.  A kept pixel's energy in every frame depends only
// on the original pixels of its 3x3 carved neighbourhood (and on its own
// original pixel in the predecessor frame for the difference term).  If the
// neighbourhood around its new position holds the same original pixels as
// the one around its old position, all its energies -- hence its key -- are
// unchanged and move with it; otherwise they are recomputed from the T
// frames (refresh_kernel).  This is exact: the result equals a full
// recomputation.

// One wavefront per row, four rows per block, no block barriers.  The
// row's seam thresholds R_s - s are staged in LDS (one slot per lane).  Per
// pass of up to 2048 new columns, the old entries they can come from (the
// same columns plus kk) are copied into the wavefront's LDS with 16-byte
// loads; a lane then builds 8 consecutive new columns in each of four
// 512-column chunks -- the count of thresholds at or below its first column
// found once, then stepped -- from LDS, and writes each chunk with 16-byte
// stores.  Rows with more than kUpdSeams seams gather their entries straight
// from global memory instead.
// Variants (rows per workgroup ROWS, new columns per pass SPAN); the
// default is (4, 2048), the others are for the batch autotuner.
constexpr int kUpdSeams = 64;                          // seams per row staged in LDS

// Compaction of row i of job J in iteration r (width Wr, kk seams): the
// column map and, when a further iteration reads them, the keys.  One
// wavefront; thr: its kUpdSeams + 1 threshold slots in LDS, holding R_s - s
// (and INT_MAX beyond) when kk <= kUpdSeams; sM, sK: its staging (SPAN +
// kUpdSeams + 8 entries each).  Rows with more seams read the thresholds
// from J.seams.
template <int SPAN>
__device__ __forceinline__ void compact_row(const Job &J, int r, int Wr, int kk, int i, const int *thr, uint16_t *sM,
                                            uint16_t *sK, int lane)
{
    static_assert(SPAN % 512 == 0, "passes of whole 512-column chunks");
    constexpr int kUpdStage = SPAN + kUpdSeams + 8;    // old entries staged per pass
    const int Wn = Wr - kk;
    const int Wp = J.Wp;
    // in place: new column j never reads an old column left of j, and every
    // entry is read before the wavefront writes over it
    int16_t *Mr = J.M + (size_t)i * Wp;
    uint16_t *Kr = J.K + (size_t)i * J.Kp + J.KL;
    const bool keys = Wn > J.Wt;  // a further iteration reads the keys
    const int16_t *__restrict__ R = J.seams + (size_t)i * J.kcap;  // removed columns of row i, increasing
    // seam s removed old column R[s]; new column j reads old column j + #{s : R[s] - s <= j}
    const bool staged = kk <= kUpdSeams;
    auto rs = [&](int s) -> int {
        if (staged) return thr[min(s, kUpdSeams)];
        return s < kk ? (int)R[s] - s : 0x7fffffff;
    };
    // the rows' first Wr entries (rounded up to whole 16-byte groups, within
    // the Wp and Kp - KL entries of the row buffers) as buffer resources: the
    // staged passes request whole groups up to SPAN + kk columns past their
    // start, and those past the current width read 0 and move no data
    const int wr8 = (Wr + 7) & ~7;
    const __amdgpu_buffer_rsrc_t rM =
        __builtin_amdgcn_make_buffer_rsrc((void *)Mr, (short)0, 2 * min(wr8, Wp), 0x00020000);
    const __amdgpu_buffer_rsrc_t rK =
        __builtin_amdgcn_make_buffer_rsrc((void *)Kr, (short)0, 2 * min(wr8, J.Kp - J.KL), 0x00020000);
    // columns left of the first threshold keep their entries: passes start at
    // the 8-aligned column below it
    const int jstart = min(rs(0), Wn) & ~7;
    // count of thresholds at or below column jb
    auto count = [&](int jb) {
        int a = 0;
        if (kk <= 32) {
            for (int s = 0; s < kk; ++s) a += rs(s) <= jb ? 1 : 0;  // same slot in every lane
        } else {
            int hi = kk;
            while (a < hi) {
                const int m = (a + hi) >> 1;
                if (rs(m) <= jb) a = m + 1;
                else hi = m;
            }
        }
        return a;
    };
    auto put = [&](int jb, const u16x2 (&mv)[4], const u16x2 (&kv)[4]) {
        if (jb + 8 <= Wn) {
            *gp(reinterpret_cast<u32x4 *>(Mr + jb)) = u32x4{pack2(mv[0]), pack2(mv[1]), pack2(mv[2]), pack2(mv[3])};
            if (keys) *gp(reinterpret_cast<u32x4 *>(Kr + jb)) = u32x4{pack2(kv[0]), pack2(kv[1]), pack2(kv[2]), pack2(kv[3])};
        } else {
            for (int q = 0; q < 8 && jb + q < Wn; ++q) {
                Mr[jb + q] = (int16_t)mv[q >> 1][q & 1];
                if (keys) Kr[jb + q] = kv[q >> 1][q & 1];
            }
        }
    };
    if (staged) {
        for (int j0 = jstart; j0 < Wn; j0 += SPAN) {
            // old columns [j0, hi) hold every source of new columns [j0, j0 + SPAN)
            const int hi = min(j0 + SPAN + kk, Wr);
            const int nv = (hi - j0 + 7) >> 3;  // 16-byte groups, within the row buffers
            // all groups requested before the first is written (a group past
            // the row buffer reads 0 and is not kept)
            constexpr int kG = (kUpdStage / 8 + 63) / 64;
            u32x4 tm[kG], tk[kG];
#pragma unroll
            for (int u = 0; u < kG; ++u) {
                const int off = 2 * (j0 + 8 * (lane + 64 * u));
                tm[u] = __builtin_amdgcn_raw_buffer_load_b128(rM, off, 0, 0);
                tk[u] = keys ? __builtin_amdgcn_raw_buffer_load_b128(rK, off, 0, 0) : u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int u = 0; u < kG; ++u) {
                const int v = lane + 64 * u;
                if (v < nv) {
                    *reinterpret_cast<u32x4 *>(sM + 8 * v) = tm[u];
                    *reinterpret_cast<u32x4 *>(sK + 8 * v) = tk[u];
                }
            }
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = 0; c < SPAN / 512; ++c) {
                const int jb = j0 + 512 * c + 8 * lane;
                if (jb >= Wn) break;
                int a = count(jb);
                int nxt = rs(a);
                u16x2 mv[4], kv[4];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int j = jb + q;
                    while (nxt <= j) nxt = rs(++a);
                    const int x = min(j + a, Wr - 1) - j0;  // columns past Wn read a staged entry, never stored
                    mv[q >> 1][q & 1] = sM[x];
                    kv[q >> 1][q & 1] = keys ? sK[x] : (uint16_t)0;
                }
                put(jb, mv, kv);
            }
            __builtin_amdgcn_wave_barrier();
        }
    } else {
        for (int jb = jstart + 8 * lane; jb < Wn; jb += 512) {
            int a = count(jb);
            int nxt = rs(a);
            u16x2 mv[4], kv[4];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = jb + q;
                while (nxt <= j) nxt = rs(++a);
                const int off = 2 * min(j + a, Wr - 1);
                mv[q >> 1][q & 1] = __builtin_amdgcn_raw_buffer_load_b16(rM, off, 0, 0);
                kv[q >> 1][q & 1] = keys ? __builtin_amdgcn_raw_buffer_load_b16(rK, off, 0, 0) : (uint16_t)0;
            }
            put(jb, mv, kv);
        }
    }
    if (!keys) return;
    // the keys of the vacated columns become 0xffff; columns beyond the
    // previous width of this buffer already are
    const int wprev = r > 0 ? J.log[4 * (r - 1)] : J.W;
    for (int j = Wn + lane; j < wprev; j += 64) Kr[j] = kRowInf;
}

template <int ROWS, int SPAN>
__global__ __launch_bounds__(64 * ROWS) void update_kernel(const Job *jobs)
{
    constexpr int kUpdStage = SPAN + kUpdSeams + 8;
    __shared__ int thr[ROWS][kUpdSeams + 1];
    __shared__ __align__(16) uint16_t stM[ROWS][kUpdStage];
    __shared__ __align__(16) uint16_t stK[ROWS][kUpdStage];
    const Job &J = jobs[blockIdx.y];
    // job state read from memory: the same in every lane
    const int r = __builtin_amdgcn_readfirstlane(job_iter(J));
    const int Wr = __builtin_amdgcn_readfirstlane(job_width(J, r));
    if (Wr <= J.Wt) return;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i = __builtin_amdgcn_readfirstlane((int)blockIdx.x * ROWS + w);
    if (i >= J.H) return;
    const int lane = threadIdx.x & 63;
    const int kk = __builtin_amdgcn_readfirstlane(J.log[4 * r + 2]);
    if (kk <= kUpdSeams) {
        const int16_t *R = J.seams + (size_t)i * J.kcap;
        thr[w][lane] = lane < kk ? (int)R[lane] - lane : 0x7fffffff;
        if (lane == 0) thr[w][kUpdSeams] = 0x7fffffff;
        __builtin_amdgcn_wave_barrier();
    }
    compact_row<SPAN>(J, r, Wr, kk, i, thr[w], stM[w], stK[w], lane);
}

// ------------------------------------------- backtrack within a band + compaction
//
// The fill and compaction of one iteration fused: one workgroup of WAVES
// wavefronts per (band of 32 rows, job).  First the seams' paths through the
// band, as fill_kernel: a wavefront stages the window of the band's
// indicator rows a seam can reach from its column at the band's last row, and
// one lane follows it upward.  Then every seam's column in every row of the
// band (for the refresh) and its removal mark in the buffer mask, through the
// column map before it moves.  Seams are taken 64 at a time.  Then the band's
// rows are compacted, as update_kernel, with their thresholds taken from the
// paths in LDS (from the seam rows just written when there are more than 64
// seams).  No row of the band needs anything from another band.  Serves jobs
// with 32-row bands.
constexpr int kFuseB = 32;
constexpr int kFuseSpan = 1024;                // new columns per compaction pass
constexpr int kFuseWin = 2 * kFuseB + 8;       // window pitch: a seam's window is at most 2 B - 1 wide, staged from a word
constexpr int kFuseStage = kFuseSpan + kUpdSeams + 8;

__host__ __device__ constexpr size_t band_update_lds(int waves)
{
    return (size_t)waves * 2 * kFuseStage * 2 +           // staged column-map and key entries, per wavefront
           (size_t)waves * (kFuseB - 1) * kFuseWin +       // seam windows, per wavefront
           (size_t)kUpdSeams * kFuseB * 2 +                // paths: column of seam s in row lo + q
           (size_t)waves * (kUpdSeams + 1) * 4;            // thresholds of the row a wavefront compacts
}

// Band b of job J in iteration r (width Wr > Wt) by 64 WAVES threads; fsm:
// band_update_lds(WAVES) bytes of LDS, 16-byte aligned.
template <int WAVES>
__device__ __forceinline__ void band_update_body(const Job &J, int r, int Wr, int b, uint8_t *fsm)
{
    uint16_t *stM = reinterpret_cast<uint16_t *>(fsm);
    uint16_t *stK = stM + (size_t)WAVES * kFuseStage;
    uint8_t *win = reinterpret_cast<uint8_t *>(stK + (size_t)WAVES * kFuseStage);
    int16_t *path = reinterpret_cast<int16_t *>(win + (size_t)WAVES * (kFuseB - 1) * kFuseWin);  // [kUpdSeams][kFuseB]
    int *thr = reinterpret_cast<int *>(path + (size_t)kUpdSeams * kFuseB);
    const int kk = __builtin_amdgcn_readfirstlane(J.log[4 * r + 2]);
    const int H = J.H, nb = J.nb, W = J.W, Wp = J.Wp;
    const int lo = b * kFuseB, hi = min(lo + kFuseB, H) - 1;
    const int span = hi - lo;  // < kFuseB
    const int rows = span + 1;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    uint8_t *ww = win + (size_t)w * (kFuseB - 1) * kFuseWin;
    for (int s0 = 0; s0 < kk; s0 += kUpdSeams) {
        const int ns = min(kUpdSeams, kk - s0);
        // 1. the paths of seams [s0, s0 + ns) through the band
        for (int s = w; s < ns; s += WAVES) {
            const int c_end = J.bcol[(s0 + s) * nb + b];
            const int wlo = max(c_end - span, 0), whi = min(c_end + span + 1, Wr);
            const int sh = stage_bytes(ww, kFuseWin, J.dir, Wp, lo + 1, span, wlo, whi, lane, 64) - wlo;
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                int c = c_end;
                path[s * kFuseB + span] = (int16_t)c;
                for (int i = hi; i > lo; --i) {
                    c += code_step(ww[(i - lo - 1) * kFuseWin + c + sh]);
                    path[s * kFuseB + i - 1 - lo] = (int16_t)c;
                }
            }
            __builtin_amdgcn_wave_barrier();  // the window is read before the next seam's staging
        }
        __syncthreads();
        // 2. their columns in every row of the band, and their marks in the
        // buffer mask (original columns, through the column map before it moves)
        for (int x = (int)threadIdx.x; x < ns * rows; x += 64 * WAVES) {
            const int s = x / rows, q = x - s * rows;
            const int i = lo + q;
            const int col = path[s * kFuseB + q];
            J.seams[(size_t)i * J.kcap + s0 + s] = (int16_t)col;
            J.bmask[(size_t)i * W + mcol(J.M + (size_t)i * Wp, col, W)] = (uint16_t)(r + 1);
        }
        __syncthreads();  // every mark has read the column map; the paths may be overwritten
    }
    // 3. the band's rows compacted
    int *tw = thr + (size_t)w * (kUpdSeams + 1);
    uint16_t *sM = stM + (size_t)w * kFuseStage, *sK = stK + (size_t)w * kFuseStage;
    for (int q = w; q < rows; q += WAVES) {
        if (kk <= kUpdSeams) {
            tw[lane] = lane < kk ? (int)path[lane * kFuseB + q] - lane : 0x7fffffff;
            if (lane == 0) tw[kUpdSeams] = 0x7fffffff;
        }
        __builtin_amdgcn_wave_barrier();
        compact_row<kFuseSpan>(J, r, Wr, kk, lo + q, tw, sM, sK, lane);
        __builtin_amdgcn_wave_barrier();  // the thresholds are read before the next row's
    }
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void band_update_kernel(const Job *jobs)
{
    extern __shared__ __align__(16) uint8_t fsm[];
    const Job &J = jobs[blockIdx.y];
    const int r = __builtin_amdgcn_readfirstlane(job_iter(J));
    const int Wr = __builtin_amdgcn_readfirstlane(job_width(J, r));
    if (Wr <= J.Wt) return;
    if ((int)blockIdx.x >= J.nb) return;
    band_update_body<WAVES>(J, r, Wr, (int)blockIdx.x, fsm);
}

// Refresh of the pixels whose 3x3 neighbourhood changed.  Column-map rows
// are strictly increasing, so two carved positions hold the same original
// pixel exactly when they map to the same old column: with R_q the removed
// old columns of row q (minus their rank), new column c of row q was old
// column c + #{s : R_q[s] <= c}.  Pixel (i, j) keeps its energy in every
// frame iff each of its 8 neighbours, taken on the new grid, was the
// matching neighbour of its old position (i, o_i(j)) on the old grid
// (borders replicated on each grid).  Only columns within 3 of a removed
// pixel of rows i-1..i+1 can fail the test.
//
// One block per (band of 16 rows, job): the candidates around every seam
// are tested, the affected ones (usually 2-4 per seam and row) listed in
// LDS, and each gets a share of the block's threads that sum its energy
// over the T frames.  Threads next to each other work on pixels of the same
// band and the same frame, so their loads share a few luma tiles.  A
// candidate also in the window of the seam on its left is left to that
// seam.

constexpr int kRefreshRows = 16;
constexpr int kRefreshList = 512;
constexpr int kRefreshSeams = 64;  // seams whose positions are staged in LDS

// NT threads per block: 256 when the launch has blocks enough to fill the
// device; 1024 when it has few (a pixel's frames then split over more
// threads, which shortens the block).
// The end of a job's iteration: the last workgroup of the launch to finish
// for a job (counted in the iteration's free log word, which the selection
// of the iteration before, or the job set-up, zeroed) moves the job's
// iteration counter on.  Every workgroup has read the counter by then, since
// each reads it first and counts itself last.  The count is a relaxed atomic
// with no fence: the next kernel sees the keys written here through the
// kernel boundary, and an agent-scope fence per workgroup would write back
// the XCD's whole L2 each time.
__device__ __forceinline__ void end_iteration(const Job &J, int r)
{
    __syncthreads();
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add(&J.log[4 * r + 3], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
            (int)gridDim.x - 1)
        J.state[3] = r + 1;
}

struct RefreshLds {
    int R[kRefreshRows + 2][kRefreshSeams];  // rows i0-1 .. i0+16 (clamped): old column - s
    int flist[kRefreshList];                 // (row in band << 16) | new column
    Stencil fst[kRefreshList];
    uint32_t fsum[kRefreshList];
    int nf;
};

// Rows [16 bx, 16 bx + 16) of job J in iteration r (width Wr > Wt) by NT
// threads, with L in LDS.
template <int NT>
__device__ __forceinline__ void refresh_body(const Job &J, int r, int Wr, int bx, RefreshLds &L)
{
    auto &R = L.R;
    auto &flist = L.flist;
    auto &fst = L.fst;
    auto &fsum = L.fsum;
    auto &nf = L.nf;
    const int kk = J.log[4 * r + 2];
    const int Wn = Wr - kk;
    const int H = J.H, Wp = J.Wp, W = J.W, T = J.T;
    const int Kp = J.Kp;
    const int i0 = bx * kRefreshRows;
    // the job's last iteration needs no refresh, nor do rows past its height,
    // but every workgroup of the job counts itself done below
    if (Wn > J.Wt && i0 < H) {
        const int nrows = min(kRefreshRows, H - i0);
        const int16_t *__restrict__ Mn = J.M;
        uint16_t *__restrict__ Kn = J.K + J.KL;
        const int tid = threadIdx.x;
        const bool rl = kk <= kRefreshSeams;
        if (tid == 0) nf = 0;
        if (rl)
            for (int idx = tid; idx < (nrows + 2) * kk; idx += NT) {
                const int ss = idx / (nrows + 2), rr = idx - ss * (nrows + 2);  // consecutive threads: same seam
                const int row = min(max(i0 - 1 + rr, 0), H - 1);
                R[rr][ss] = J.seams[(size_t)row * J.kcap + ss] - ss;
            }
        __syncthreads();
        // seam positions (old column - rank) of row `row` (absolute, clamped)
        auto rsd = [&](int row, int ss) -> int {
            row = min(max(row, 0), H - 1);
            return rl ? R[row - (i0 - 1)][ss] : (int)J.seams[(size_t)row * J.kcap + ss] - ss;
        };
        // old column of new column c in row `row`
        auto oldcol = [&](int row, int c) -> int {
            int a = 0, b = kk;
            while (a < b) {
                const int m = (a + b) >> 1;
                if (rsd(row, m) <= c) a = m + 1;
                else b = m;
            }
            return c + a;
        };
        auto full_sum = [&](const Stencil &st) { return seq_sum(J, st, 0, 1); };
        // candidates: (seam, row in band, slot) triples; windows are at most 9 wide
        const int ncand = kk * nrows * 9;
        for (int u = tid; u < ncand; u += NT) {
            const int s = u / (nrows * 9);
            const int rem = u - s * (nrows * 9);
            const int rb = rem / 9, slot = rem - rb * 9;
            const int i = i0 + rb;
            const int a0 = rsd(i - 1, s), a1 = rsd(i, s), a2 = rsd(i + 1, s);
            const int lo = max(min(min(a0, a1), a2) - 3, 0);
            const int hi = min(max(max(a0, a1), a2) + 3, Wn - 1);
            const int c = lo + slot;
            if (c > hi) continue;
            if (s > 0 && c <= max(max(rsd(i - 1, s - 1), rsd(i, s - 1)), rsd(i + 1, s - 1)) + 3) continue;
            const int src = oldcol(i, c);
            bool same = true;
    #pragma unroll
            for (int dq = -1; dq <= 1; ++dq)
    #pragma unroll
                for (int dj = -1; dj <= 1; ++dj) {
                    if (dq == 0 && dj == 0) continue;
                    const int cn = min(max(c + dj, 0), Wn - 1);
                    const int co = min(max(src + dj, 0), Wr - 1);
                    same = same && oldcol(i + dq, cn) == co;
                }
            if (!same) {
                const int idx = atomicAdd(&nf, 1);
                if (idx < kRefreshList) {
                    flist[idx] = (rb << 16) | c;
                } else {  // list full: this thread does the pixel alone
                    const int im = max(i - 1, 0), ip = min(i + 1, H - 1);
                    const Stencil st = stencil_from_rows(Mn + (size_t)im * Wp, Mn + (size_t)i * Wp,
                                                         Mn + (size_t)ip * Wp, im, i, ip, c, Wn, W);
                    Kn[(size_t)i * Kp + c] = (uint16_t)((full_sum(st) / (uint32_t)T) << 2);
                }
            }
        }
        __syncthreads();
        const int n = min(nf, kRefreshList);
        for (int p = tid; p < n; p += NT) {
            const int i = i0 + (flist[p] >> 16), c = flist[p] & 0xffff;
            const int im = max(i - 1, 0), ip = min(i + 1, H - 1);
            fst[p] = stencil_from_rows(Mn + (size_t)im * Wp, Mn + (size_t)i * Wp, Mn + (size_t)ip * Wp, im, i, ip, c,
                                       Wn, W);
            fsum[p] = 0;
        }
        __syncthreads();
        if (n > 0) {
            // a wavefront takes 64 listed pixels and every tpp-th chunk of 16
            // frames
            const int ng = (n + 63) >> 6, nw = NT >> 6;
            const int tpp = max(nw / ng, 1);
            const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
            for (int task = w; task < ng * tpp; task += nw) {
                const int p = (task % ng) * 64 + (tid & 63), sub = task / ng;
                if (p < n) {
                    const Stencil st = fst[p];
                    atomicAdd(&fsum[p], seq_sum(J, st, sub, tpp));
                }
            }
        }
        __syncthreads();
        for (int p = tid; p < n; p += NT) {
            const int i = i0 + (flist[p] >> 16), c = flist[p] & 0xffff;
            Kn[(size_t)i * Kp + c] = (uint16_t)((fsum[p] / (uint32_t)T) << 2);
        }
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void refresh_kernel(const Job *jobs)
{
    __shared__ RefreshLds L;
    const Job &J = jobs[blockIdx.y];
    const int r = job_iter(J);
    const int Wr = job_width(J, r);
    if (Wr <= J.Wt) return;  // finished before this iteration: no iteration to end
    refresh_body<NT>(J, r, Wr, (int)blockIdx.x, L);
    end_iteration(J, r);
}

// ------------------------------------------------------ persistent launch
//
// Every iteration of every job of a batch in one launch.  Workgroups of 256
// threads take work items from rings in device memory; an item is one phase
// of one job's iteration, or one part of it:
//   DP        a workgroup's columns of a chunk of R rows (dp_chunk_body),
//             chunk after chunk;
//   BORG      one band's origins over 512 columns;
//   SELECT    the job's selection (one item);
//   BAND      one band's seam trace and compaction (band_update_body);
//   REFRESH   16 rows of the partial energy refresh.
// Each job counts the finished items of its current phase; the workgroup
// that finishes the last one puts the next phase's items in the job's ring
// (after the last band of a job's last iteration: the job is done).  So every
// job runs its own iteration chain, and the jobs fill the device between
// them.
//
// XCD-local mode (LOCAL): there is one ring per XCD; each job belongs to one
// ring, and only the workgroups running on that XCD (hardware register
// XCC_ID) take its items.  All of a job's reads and writes then meet in that
// XCD's L2 cache: a workgroup publishes its results by waiting until its
// stores have reached the L2 (no L2 write-back), and a workgroup that takes
// an item makes an agent-scope acquire (its L1 forgets what it holds).
// Agent mode: one ring served by every workgroup, with agent-scope release
// (L2 write-back) and acquire around every item, for devices where the XCD
// of a workgroup cannot be trusted.
//
// Ring slot t holds an item and its generation t; a workgroup takes the next
// slot number of its ring and waits until that generation appears.  It
// leaves when no job of its ring is carving, or when it has waited longer
// than wait_ticks of the wall clock (then it raises the abort flag, every
// workgroup leaves and the host reports an error): no wait is unbounded.

enum : int { kPDp = 0, kPBorg = 1, kPSelect = 2, kPBand = 3, kPRefresh = 4 };
constexpr int kPBorgCols = 512;  // columns of one band-origin item

__device__ __forceinline__ unsigned long long p_make(int job, int phase, int x)
{
    return ((unsigned long long)(unsigned)job << 32) | ((unsigned long long)(unsigned)phase << 24) |
           (unsigned long long)(unsigned)(x & 0xffffff);
}

// items of a phase of job J at width Wr (DP: per chunk)
__device__ __forceinline__ int p_items(const Job &J, int phase, int Wr, int P)
{
    switch (phase) {
    case kPDp: return (Wr + P - 1) / P;
    case kPBorg: return J.nb * ((Wr + kPBorgCols - 1) / kPBorgCols);
    case kPBand: return J.nb;
    case kPSelect: return 1;
    default: return (J.H + kRefreshRows - 1) / kRefreshRows;
    }
}

__device__ __forceinline__ int p_load(const int *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ void p_store(int *p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Waits until this wavefront's global stores have reached the L2 cache
// (s_waitcnt vmcnt(0)).  A workgroup barrier waits only for LDS, so each
// wavefront waits for its own stores before the barrier after which the
// workgroup's results count as published.
__device__ __forceinline__ void p_stores_done() { __builtin_amdgcn_s_waitcnt(0x0f70); }

// A value another workgroup wrote with an ordinary store: LOCAL, an ordinary
// load (after p_acquire_wave: it reads this XCD's L2, where the store is);
// agent mode, after the agent-scope acquire, any load.
template <bool LOCAL>
__device__ __forceinline__ int p_read(const int *p)
{
    if constexpr (LOCAL) return *p;
    else return p_load(p);
}

// Before a wavefront reads what other workgroups published: an agent-scope
// acquire, which invalidates the compute unit's L1 (and the L2's lines of
// memory that is not this XCD's to cache; in LOCAL mode the data it reads
// were written on this XCD and sit in its L2 or in memory).
template <bool LOCAL>
__device__ __forceinline__ void p_acquire_wave()
{
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Everything the workgroup wrote is published: every wavefront's stores
// reach the L2; in agent mode thread 0 then writes the L2 back.
template <bool LOCAL>
__device__ __forceinline__ void p_release_block()
{
    p_stores_done();
    __syncthreads();
    if constexpr (!LOCAL) {
        if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
}

struct PRing {
    PState *st;
    unsigned long long *seq, *item;
};

__device__ __forceinline__ PRing p_ring(const PArgs &a, int ring)
{
    const size_t cap = (size_t)a.cap_mask + 1;
    return PRing{a.st + ring, a.seq + (size_t)ring * cap, a.item + (size_t)ring * cap};
}

// n items (job, phase, xf(i)) into ring q, by the whole workgroup; what
// every thread wrote before is published with them.
template <bool LOCAL, class XF>
__device__ void p_push(const PArgs &a, const PRing &q, int job, int phase, int n, XF xf, int *s_t0)
{
    if (threadIdx.x == 0) *s_t0 = __hip_atomic_fetch_add(&q.st->tail, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int t0 = *s_t0;
    for (int i = threadIdx.x; i < n; i += kPersistThreads)
        q.item[(unsigned)(t0 + i) & a.cap_mask] = p_make(job, phase, xf(i));
    p_release_block<LOCAL>();
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kPersistThreads)
        __hip_atomic_store(&q.seq[(unsigned)(t0 + i) & a.cap_mask], (unsigned long long)(unsigned)(t0 + i),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A job's iteration ends: it moves to iteration r + 1 and carves on (its DP
// items), or it is done.
template <bool LOCAL>
__device__ void p_end_iteration(const PArgs &a, const PRing &q, const Job &J, int job, int r, int Wn, int *s_t0)
{
    if (threadIdx.x == 0) p_store(&J.state[3], r + 1);
    if (Wn > J.Wt) {
        if (r + 2 >= J.logcap) {  // every iteration removes a column: cannot happen
            if (threadIdx.x == 0) p_store(&a.st->abort, 1);
            return;
        }
        p_push<LOCAL>(a, q, job, kPDp, (Wn + a.P - 1) / a.P, [](int i) { return i; }, s_t0);
        return;
    }
    p_stores_done();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_fetch_add(&q.st->active, -1, LOCAL ? __ATOMIC_RELAXED : __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
}

template <bool LOCAL>
__global__ __launch_bounds__(kPersistThreads, 4) void persist_kernel(PArgs a)
{
    extern __shared__ __align__(16) uint8_t psm[];
    __shared__ unsigned long long s_item;
    __shared__ int s_flag, s_t0;
    __shared__ int scan_tmp[16];
    __shared__ unsigned long long tr[kPTrace];  // this workgroup's trace counters (thread 0)
    const int tid = threadIdx.x;
    if (tid < kPTrace) tr[tid] = 0;
    // the ring this workgroup serves: its XCD's (LOCAL), or the only one
    int ring = 0;
    if constexpr (LOCAL) ring = a.xcc_ring[__builtin_amdgcn_s_getreg((3 << 11) | 20) & 15];  // XCC_ID[3:0]
    ring = __builtin_amdgcn_readfirstlane(ring);
    if (ring < 0 || ring >= a.nring) return;  // an XCD with no ring: nothing to take
    const PRing q = p_ring(a, ring);
    for (;;) {
        // take the next slot and wait for its item
        if (tid == 0) {
            const long long w0 = a.trace ? (long long)wall_clock64() : 0;
            const int t = __hip_atomic_fetch_add(&q.st->head, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long want = (unsigned long long)(unsigned)t;
            const unsigned long long *sp = q.seq + ((unsigned)t & a.cap_mask);
            const long long t_start = (long long)wall_clock64();
            int stop = 0;
            for (unsigned spins = 0;; ++spins) {
                if (__hip_atomic_load(sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want) break;
                if ((spins & 7) == 7) {
                    if (p_load(&q.st->active) == 0 || p_load(&a.st->abort) != 0) {
                        stop = 1;
                        break;
                    }
                    if ((long long)wall_clock64() - t_start > a.wait_ticks) {
                        p_store(&a.st->abort, 1);
                        stop = 1;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(4);
            }
            if (!stop) {
                p_acquire_wave<LOCAL>();
                if constexpr (LOCAL) s_item = q.item[(unsigned)t & a.cap_mask];
                else s_item = __hip_atomic_load(q.item + ((unsigned)t & a.cap_mask), __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
            }
            s_flag = stop;
            if (a.trace) {
                tr[kPTraceWait] += (unsigned long long)((long long)wall_clock64() - w0);
                tr[kPTraceWait + 1] += 1;
            }
        }
        __syncthreads();
        if (s_flag) {
            if (tid == 0 && a.trace)
                for (int k = 0; k < kPTrace; ++k)
                    if (tr[k]) __hip_atomic_fetch_add(&a.trace[k], tr[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        if (tid >= 64) p_acquire_wave<LOCAL>();
        const long long b0 = (tid == 0 && a.trace) ? (long long)wall_clock64() : 0;
        const unsigned long long it = s_item;
        const int job = __builtin_amdgcn_readfirstlane((int)(it >> 32));
        const int phase = __builtin_amdgcn_readfirstlane((int)((it >> 24) & 0xff));
        const int x = __builtin_amdgcn_readfirstlane((int)(it & 0xffffff));
        const Job &J = a.jobs[job];
        const int r = __builtin_amdgcn_readfirstlane(p_load(&J.state[3]));
        const int Wr = __builtin_amdgcn_readfirstlane(r < J.logcap ? p_read<LOCAL>(&J.log[4 * r]) : J.Wt);
        switch (phase) {
        case kPDp:
            dp_chunk_body<4, 16, 8>(J, Wr, x & 0xfff, (x >> 12) * a.R, a.R, a.P, kPersistThreads,
                                    reinterpret_cast<uint32_t *>(psm));
            break;
        case kPBorg: {
            const int cg = x >> 12;  // column group of kPBorgCols columns
            for (int c0 = cg * kPBorgCols; c0 < min((cg + 1) * kPBorgCols, Wr); c0 += kPersistThreads) {
                borg_body<kPersistThreads>(J, Wr, x & 0xfff, c0, psm);
                __syncthreads();  // the tile is read before the next columns are staged
            }
            break;
        }
        case kPSelect:
            select_body<kPersistThreads>(J, r, Wr, a.sel_lds, 0, reinterpret_cast<uint64_t *>(psm), scan_tmp);
            break;
        case kPBand: band_update_body<kPersistThreads / 64>(J, r, Wr, x, psm); break;
        default: refresh_body<kPersistThreads>(J, r, Wr, x, *reinterpret_cast<RefreshLds *>(psm)); break;
        }
        // count the item done; the last of its phase starts the next phase
        const long long b1 = (tid == 0 && a.trace) ? (long long)wall_clock64() : 0;
        p_stores_done();
        __syncthreads();
        if (tid == 0) {
            const int n = p_items(J, phase, Wr, a.P);
            const int old = __hip_atomic_fetch_add(&a.cnt[job], 1, LOCAL ? __ATOMIC_RELAXED : __ATOMIC_ACQ_REL,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            s_flag = old == n - 1;
            if (old == n - 1) p_store(&a.cnt[job], 0);
        }
        __syncthreads();
        if (s_flag) {
            if (LOCAL || tid >= 64) p_acquire_wave<LOCAL>();
            switch (phase) {
            case kPDp: {
                const int ci = x >> 12;
                if ((ci + 1) * a.R < J.H) {
                    p_push<LOCAL>(a, q, job, kPDp, (Wr + a.P - 1) / a.P, [ci](int i) { return ((ci + 1) << 12) | i; },
                                  &s_t0);
                } else {
                    const int nb = J.nb;
                    p_push<LOCAL>(a, q, job, kPBorg, nb * ((Wr + kPBorgCols - 1) / kPBorgCols),
                                  [nb](int i) { return ((i / nb) << 12) | (i % nb); }, &s_t0);
                }
                break;
            }
            case kPBorg: p_push<LOCAL>(a, q, job, kPSelect, 1, [](int i) { return i; }, &s_t0); break;
            case kPSelect: p_push<LOCAL>(a, q, job, kPBand, J.nb, [](int i) { return i; }, &s_t0); break;
            case kPBand: {
                const int Wn = Wr - __builtin_amdgcn_readfirstlane(p_read<LOCAL>(&J.log[4 * r + 2]));
                if (Wn > J.Wt)
                    p_push<LOCAL>(a, q, job, kPRefresh, (J.H + kRefreshRows - 1) / kRefreshRows,
                                  [](int i) { return i; }, &s_t0);
                else p_end_iteration<LOCAL>(a, q, J, job, r, Wn, &s_t0);
                break;
            }
            default: {
                const int Wn = Wr - __builtin_amdgcn_readfirstlane(p_read<LOCAL>(&J.log[4 * r + 2]));
                p_end_iteration<LOCAL>(a, q, J, job, r, Wn, &s_t0);
                break;
            }
            }
        }
        if (tid == 0 && a.trace) {
            const long long b2 = (long long)wall_clock64();
            tr[2 * phase] += (unsigned long long)(b1 - b0);
            tr[2 * phase + 1] += 1;
            tr[kPTraceDone] += (unsigned long long)(b2 - b1);
        }
        __syncthreads();  // s_flag, s_t0 and s_item are read before the next item overwrites them
    }
}

// Empties the rings (every generation unset), the phase counters and the
// ring states.
__global__ __launch_bounds__(256) void persist_clear_kernel(PArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int nslots = a.nring * (a.cap_mask + 1);
    if (i < nslots) a.seq[i] = ~0ull;
    if (i < a.njobs) a.cnt[i] = 0;
    if (i < a.nring) {
        a.st[i].head = 0;
        a.st[i].tail = 0;
        a.st[i].active = 0;
        a.st[i].abort = 0;
    }
}

// The first DP chunk of every job that has columns to remove, in its ring.
__global__ __launch_bounds__(64) void persist_seed_kernel(PArgs a)
{
    if (threadIdx.x != 0) return;
    for (int j = 0; j < a.njobs; ++j) {
        const Job &J = a.jobs[j];
        const int Wr = J.log[0];
        if (Wr <= J.Wt) continue;
        const PRing q = p_ring(a, J.ring);
        const int n = (Wr + a.P - 1) / a.P;
        for (int i = 0; i < n; ++i) {
            const int t = q.st->tail++;
            q.item[(unsigned)t & a.cap_mask] = p_make(j, kPDp, i);
            q.seq[(unsigned)t & a.cap_mask] = (unsigned long long)(unsigned)t;
        }
        q.st->active += 1;
    }
}

// The XCD (hardware register XCC_ID) of every workgroup of a launch.
__global__ __launch_bounds__(64) void xcc_probe_kernel(int *out)
{
    if (threadIdx.x == 0) out[blockIdx.x] = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15;
}

// ----------------------------------------------------------------- gather
//
// Carved output of every frame of the buffer: out(t, i, j) = frame(t, i,
// M(i, j)) for j < Wt, all channels; masks of every frame = buffer mask.

// Staged form, when FPB source rows and the offsets of the output row fit
// the launch's LDS: the byte offsets of the output row within the source row
// are computed once per row, then for every FPB frames of the buffer their
// source rows are loaded into LDS with coalesced 16-byte loads (all requested
// before any is used) and the output rows are assembled from them and written
// with 16-byte stores.  Otherwise the row gathers directly.
constexpr size_t kGatherLds = 65536;  // LDS a gather workgroup may take

__device__ __forceinline__ uint32_t div3(uint32_t x) { return __umulhi(x, 0xAAAAAAABu) >> 1; }

template <int FPB>
__device__ void gather_body(const Job &J, int i, int lds_bytes, uint8_t *gsm)
{
    const int16_t *__restrict__ M = J.M + (size_t)i * J.Wp;
    const int C = J.C, W = J.W, Wt = J.Wt, H = J.H;
    const int inb = W * C, outb = Wt * C;
    const int ip = (inb + 15) & ~15;  // LDS pitch of a staged source row
    const int tid = threadIdx.x;
    const uint16_t *msrc = J.bmask + (size_t)i * W;
    const bool vmask = J.masks && ((((uintptr_t)J.masks) | (uintptr_t)(2 * W)) & 15) == 0;
    auto copy_mask = [&](int t) {
        uint16_t *mdst = J.masks + ((size_t)t * H + i) * W;
        if (vmask) {
            for (int q = tid; q < W / 8; q += 256)
                gp(reinterpret_cast<u32x4 *>(mdst))[q] = gp(reinterpret_cast<const u32x4 *>(msrc))[q];
        } else {
            for (int j = tid; j < W; j += 256) mdst[j] = msrc[j];
        }
    };
    if ((size_t)FPB * ip + 2 * (size_t)outb > (size_t)lds_bytes) {
        for (int t = J.t0; t < J.t0 + J.T; ++t) {
            const uint8_t *src = J.frames + ((size_t)t * H + i) * inb;
            uint8_t *dst = J.out + ((size_t)t * H + i) * outb;
            for (int b = tid; b < outb; b += 256) {
                const int j = C == 1 ? b : (int)div3((uint32_t)b);
                dst[b] = src[mcol(M, j, W) * C + (b - j * C)];
            }
            if (J.masks) copy_mask(t);
        }
        return;
    }
    uint8_t *srow = gsm;
    uint16_t *ofs = reinterpret_cast<uint16_t *>(gsm + (size_t)FPB * ip);
    for (int b = tid; b < outb; b += 256) {
        const int j = C == 1 ? b : (int)div3((uint32_t)b);
        ofs[b] = (uint16_t)(mcol(M, j, W) * C + (b - j * C));
    }
    const bool vin = ((((uintptr_t)J.frames) | (uintptr_t)inb) & 15) == 0;
    const bool vout = ((((uintptr_t)J.out) | (uintptr_t)outb) & 15) == 0;
    const int q16 = inb / 16;
    for (int t0 = J.t0; t0 < J.t0 + J.T; t0 += FPB) {
        const int nf = min(FPB, J.t0 + J.T - t0);
        __syncthreads();  // offsets written; the previous frames' reads of the rows done
        if (vin) {
            constexpr int kReq = 4;  // 16-byte loads per thread and frame held before any is stored
#pragma unroll
            for (int f = 0; f < FPB; ++f) {
                if (f >= nf) break;
                const u32x4 *src = reinterpret_cast<const u32x4 *>(J.frames + ((size_t)(t0 + f) * H + i) * inb);
                u32x4 *dst = reinterpret_cast<u32x4 *>(srow + (size_t)f * ip);
                for (int q0 = tid; q0 < q16; q0 += 256 * kReq) {
                    u32x4 v[kReq];
#pragma unroll
                    for (int u = 0; u < kReq; ++u) {
                        const int q = q0 + 256 * u;
                        if (q < q16) v[u] = gp(src)[q];
                    }
#pragma unroll
                    for (int u = 0; u < kReq; ++u) {
                        const int q = q0 + 256 * u;
                        if (q < q16) dst[q] = v[u];
                    }
                }
            }
        } else {
            for (int f = 0; f < nf; ++f) {
                const uint8_t *src = J.frames + ((size_t)(t0 + f) * H + i) * inb;
                for (int b = tid; b < inb; b += 256) srow[(size_t)f * ip + b] = gp(src)[b];
            }
        }
        __syncthreads();
        for (int f = 0; f < nf; ++f) {
            const uint8_t *sr = srow + (size_t)f * ip;
            uint8_t *dst = J.out + ((size_t)(t0 + f) * H + i) * outb;
            if (vout) {
                for (int q = tid; q < outb / 16; q += 256) {
                    const u32x4 oa = reinterpret_cast<const u32x4 *>(ofs)[2 * q];
                    const u32x4 ob = reinterpret_cast<const u32x4 *>(ofs)[2 * q + 1];
                    const uint32_t o[8] = {oa.x, oa.y, oa.z, oa.w, ob.x, ob.y, ob.z, ob.w};
                    uint32_t w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t p0 = o[2 * k], p1 = o[2 * k + 1];
                        w[k] = (uint32_t)sr[p0 & 0xffff] | ((uint32_t)sr[p0 >> 16] << 8) |
                               ((uint32_t)sr[p1 & 0xffff] << 16) | ((uint32_t)sr[p1 >> 16] << 24);
                    }
                    gp(reinterpret_cast<u32x4 *>(dst))[q] = u32x4{w[0], w[1], w[2], w[3]};
                }
            } else {
                for (int b = tid; b < outb; b += 256) dst[b] = sr[ofs[b]];
            }
            if (J.masks) copy_mask(t0 + f);
        }
    }
}

template <int FPB>
__global__ __launch_bounds__(256) void gather_kernel(const Job *jobs, int lds_bytes)
{
    extern __shared__ __align__(16) uint8_t gsm[];
    const Job &J = jobs[blockIdx.y];
    const int i = blockIdx.x;
    if (i >= J.H) return;
    gather_body<FPB>(J, i, lds_bytes, gsm);
}

// The gather of a row streamed over its frames by two kinds of wavefront.
// Waves 0-1 load the source row D frames ahead into registers (KL 16-byte
// loads per lane and frame) and write each frame's row into one of two LDS
// rows; waves 2-3 assemble the output row (and copy the mask row, staged in
// LDS once) from the LDS row of the frame before and store it.  gfx9's
// vmcnt counts loads and stores alike, so a wave that did both would wait
// for its stores before each frame's loads; here loaders wait only for
// loads and storers never wait.  Every load takes a clamped frame and
// offset, so each loader issues the same loads every frame (the compiler
// can then wait for exactly the oldest frame's).  Rows not 16-byte aligned,
// wider than 128 KL 16-byte pieces, or that do not fit the LDS gather as in
// gather_kernel<1>.
template <int KL, int D>
__global__ __launch_bounds__(256) void gather_stream_kernel(const Job *jobs, int lds_bytes)
{
    extern __shared__ __align__(16) uint8_t gsm[];
    const Job &J = jobs[blockIdx.y];
    const int i = blockIdx.x;
    if (i >= J.H) return;
    const int C = J.C, W = J.W, Wt = J.Wt, H = J.H;
    const int inb = W * C, outb = Wt * C;
    const int ip = (inb + 15) & ~15;
    const int q16 = inb / 16, o16 = outb / 16;
    const int mrow = J.masks ? ((2 * W + 15) & ~15) : 0;
    const bool aligned = ((((uintptr_t)J.frames) | ((uintptr_t)J.out) | (uintptr_t)inb | (uintptr_t)outb) & 15) == 0 &&
                         (!J.masks || ((((uintptr_t)J.masks) | (uintptr_t)(2 * W)) & 15) == 0);
    if (!aligned || q16 > 128 * KL || 2 * (size_t)ip + 2 * (size_t)outb + (size_t)mrow > (size_t)lds_bytes) {
        gather_body<1>(J, i, lds_bytes, gsm);
        return;
    }
    // the job's fields in registers: stores through out and masks could
    // alias the job table, which would make every frame reload them
    const uint8_t *const frames = uniform_ptr(J.frames);
    uint8_t *const out = uniform_ptr(J.out);
    uint16_t *const masks = J.masks ? uniform_ptr(J.masks) : nullptr;
    uint8_t *srow = gsm;                                                  // 2 x ip
    uint16_t *ofs = reinterpret_cast<uint16_t *>(gsm + 2 * (size_t)ip);  // outb
    u32x4 *mk = reinterpret_cast<u32x4 *>(gsm + 2 * (size_t)ip + 2 * (size_t)outb);
    const int16_t *__restrict__ M = J.M + (size_t)i * J.Wp;
    const int tid = threadIdx.x;
    for (int b = tid; b < outb; b += 256) {
        const int j = C == 1 ? b : (int)div3((uint32_t)b);
        ofs[b] = (uint16_t)(mcol(M, j, W) * C + (b - j * C));
    }
    if (masks) {
        const u32x4 *msrc = reinterpret_cast<const u32x4 *>(J.bmask + (size_t)i * W);
        for (int q = tid; q < 2 * W / 16; q += 256) mk[q] = gp(msrc)[q];
    }
    const int t0 = J.t0, T = J.T;
    const bool loader = tid < 128;  // waves 0 and 1
    const int lt = tid & 127;
    u32x4 v[D][KL];
    auto load = [&](u32x4(&r)[KL], int t) {
        const u32x4 *src = reinterpret_cast<const u32x4 *>(frames + ((size_t)min(t, t0 + T - 1) * H + i) * inb);
#pragma unroll
        for (int u = 0; u < KL; ++u) r[u] = gp(src)[min(lt + 128 * u, q16 - 1)];
    };
    auto put = [&](const u32x4(&r)[KL], int b) {
        u32x4 *dst = reinterpret_cast<u32x4 *>(srow + (size_t)b * ip);
#pragma unroll
        for (int u = 0; u < KL; ++u)
            if (lt + 128 * u < q16) dst[lt + 128 * u] = r[u];
    };
    if (loader) {
#pragma unroll
        for (int d = 0; d < D; ++d) load(v[d], t0 + d);
        put(v[0], 0);
        load(v[0], t0 + D);
    }
    __syncthreads();  // offsets, mask row, frame 0's row
    // Two loops, one per kind of wavefront, with one barrier per frame each
    // (waves 0-1 take the first, 2-3 the second: the branch is uniform in
    // every wavefront), so that the compiler counts each kind's memory
    // operations apart.
    if (loader) {
        for (int f = 0; f < T; f += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                if (f + d >= T) break;
                // frame f + d + 1 into the LDS row the storers left at the
                // last barrier; its set reloads D frames ahead
                put(v[(d + 1) % D], (f + d + 1) & 1);
                load(v[(d + 1) % D], t0 + f + d + 1 + D);
                __syncthreads();
            }
        }
    } else {
        const int st = tid - 128;
        for (int f = 0; f < T; f += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int ff = f + d;
                if (ff >= T) break;
                const uint8_t *sr = srow + (size_t)(ff & 1) * ip;
                u32x4 *dst = reinterpret_cast<u32x4 *>(out + ((size_t)(t0 + ff) * H + i) * outb);
                for (int q = st; q < o16; q += 128) {
                    const u32x4 oa = reinterpret_cast<const u32x4 *>(ofs)[2 * q];
                    const u32x4 ob = reinterpret_cast<const u32x4 *>(ofs)[2 * q + 1];
                    const uint32_t o[8] = {oa.x, oa.y, oa.z, oa.w, ob.x, ob.y, ob.z, ob.w};
                    uint32_t w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint32_t p0 = o[2 * k], p1 = o[2 * k + 1];
                        w[k] = (uint32_t)sr[p0 & 0xffff] | ((uint32_t)sr[p0 >> 16] << 8) |
                               ((uint32_t)sr[p1 & 0xffff] << 16) | ((uint32_t)sr[p1 >> 16] << 24);
                    }
                    gp(dst)[q] = u32x4{w[0], w[1], w[2], w[3]};
                }
                if (masks) {
                    u32x4 *mdst = reinterpret_cast<u32x4 *>(masks + ((size_t)(t0 + ff) * H + i) * W);
                    for (int q = st; q < 2 * W / 16; q += 128) gp(mdst)[q] = mk[q];
                }
                __syncthreads();  // frame ff's row read; frame ff + 1's row written
            }
        }
    }
}

// ---------------------------------------------------------- transposes
//
// Height retargeting carves the transposed frames.  dst[n][w][h] = src[n][h][w]
// for elements of E bytes (a pixel of C channels, or a 16-bit mask entry);
// a block moves a 32 x 32 tile through LDS so both sides are read and
// written along rows.

template <int E>
__global__ __launch_bounds__(256) void transpose_kernel(const uint8_t *__restrict__ src, int H, int W,
                                                        uint8_t *__restrict__ dst)
{
    __shared__ uint8_t tile[32][32 * E + 4];
    const size_t n = blockIdx.z;
    const int h0 = blockIdx.y * 32, w0 = blockIdx.x * 32;
    const uint8_t *s = src + n * H * (size_t)W * E;
    uint8_t *d = dst + n * H * (size_t)W * E;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int h = h0 + r, w = w0 + tx;
        if (h < H && w < W)
#pragma unroll
            for (int e = 0; e < E; ++e) tile[r][tx * E + e] = s[((size_t)h * W + w) * E + e];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int w = w0 + r, h = h0 + tx;
        if (h < H && w < W)
#pragma unroll
            for (int e = 0; e < E; ++e) d[((size_t)w * H + h) * E + e] = tile[tx][r * E + e];
    }
}

// -------------------------------------------------- one-frame compaction
//
// Stage entry point of the one-pass removal (Sec. 3.1): row i of an H x W x
// C frame loses the kk columns seams[s * H + i] (increasing in s); new
// column j reads old column j + #{s : seams[s] - s <= j}.  One block per
// row; the row's seam positions are staged in LDS when there are few.

constexpr int kCompactSeams = 1024;

__global__ __launch_bounds__(256) void compact_frame_kernel(const uint8_t *in, int H, int W, int C, const int32_t *seams,
                                                            int kk, uint8_t *out)
{
    __shared__ int R[kCompactSeams];
    const int i = blockIdx.x;
    const bool lds = kk <= kCompactSeams;
    if (lds)
        for (int s = threadIdx.x; s < kk; s += 256) R[s] = seams[(size_t)s * H + i] - s;
    __syncthreads();
    auto rs = [&](int s) { return lds ? R[s] : seams[(size_t)s * H + i] - s; };
    const int Wn = W - kk;
    const uint8_t *src = in + (size_t)i * W * C;
    uint8_t *dst = out + (size_t)i * Wn * C;
    for (int j = threadIdx.x; j < Wn; j += 256) {
        int a = 0, b = kk;
        while (a < b) {
            const int m = (a + b) >> 1;
            if (rs(m) <= j) a = m + 1;
            else b = m;
        }
        const int o = min(max(j + a, 0), W - 1);
        for (int c = 0; c < C; ++c) dst[(size_t)j * C + c] = src[(size_t)o * C + c];
    }
}

// ------------------------------------------------- stage-API conversions

// U -> key row entry; *bad is set when some U lies outside [0, 16382] (the
// caller then runs no DP on the keys)
__global__ void u_to_keys_kernel(const int32_t *src, uint16_t *dst, int H, int W, int pitch, int32_t *bad)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p - (int64_t)i * W);
    const int32_t u = src[p];
    if ((uint32_t)u > 16382u) atomicOr(bad, 1);
    dst[(size_t)i * pitch + j] = (uint16_t)((uint32_t)u << 2);
}

__global__ void keys_to_u_kernel(const uint16_t *src, int32_t *dst, int H, int W, int pitch)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p - (int64_t)i * W);
    dst[p] = (int32_t)(src[(size_t)i * pitch + j] >> 2);
}

// seams (row-major, H x pitch) -> kk x H int32
__global__ void seams_out_kernel(const int16_t *src, int pitch, int32_t *dst, int kk, int H)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)kk * H) return;
    const int s = (int)(p / H), i = (int)(p - (int64_t)s * H);
    dst[p] = src[(size_t)i * pitch + s];
}

__global__ void dir_out_kernel(const uint8_t *codes, int pitch, int8_t *dst, int H, int W)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p - (int64_t)i * W);
    dst[p] = (int8_t)((int)(codes[(size_t)i * pitch + j] & 3u) - 1);
}

__global__ void dir_in_kernel(const int8_t *src, uint8_t *codes, int pitch, int H, int W)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p - (int64_t)i * W);
    const int d = src[p];
    codes[(size_t)i * pitch + j] = (uint8_t)(min(max(d, -1), 1) + 1);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------- launchers

void launch_tile_luma(const uint8_t *src, int C, int N, int H, int W, uint8_t *dst, hipStream_t s)
{
    const int vec = (W % kTileW == 0) && ((((uintptr_t)src) & 7) == 0);
    const dim3 g((unsigned)((int64_t)N * ((H + 15) / 16)), blocks_for(W, 128));
    hipLaunchKernelGGL(tile_luma_kernel, g, dim3(256), 0, s, src, C, N, H, W, dst, vec);
}

void launch_seq(const uint8_t *tiled, int N, int H, int W, uint8_t *seq, int seqp, hipStream_t s)
{
    const int ntc = tiles_across(W);
    const int tiles = ((H + kTileH - 1) / kTileH) * ntc;
    hipLaunchKernelGGL(seq_kernel, dim3(tiles), dim3(128), 0, s, tiled, N, H, W, tiled_frame_bytes(H, W), ntc, seq,
                       seqp);
}

void launch_untile(const uint8_t *src, int N, int H, int W, uint8_t *dst, hipStream_t s)
{
    hipLaunchKernelGGL(untile_kernel, dim3(blocks_for((int64_t)N * H * W, 256)), dim3(256), 0, s, src, N, H, W, dst);
}

void launch_luma(const uint8_t *rgb, uint8_t *y, int64_t npx, hipStream_t s)
{
    if (npx <= 0) return;
    if ((((uintptr_t)rgb) | ((uintptr_t)y)) & 15)
        hipLaunchKernelGGL(luma_scalar_kernel, dim3(blocks_for(npx, 256)), dim3(256), 0, s, rgb, y, npx);
    else
        hipLaunchKernelGGL(luma_vec_kernel, dim3(blocks_for(npx, 256 * 16)), dim3(256), 0, s, rgb, y, npx);
}

void launch_seg_windows(const SegArgs *d_args, int n, int ntc_max, int Hmax, hipStream_t s)
{
    hipLaunchKernelGGL(seg_window_kernel, dim3(blocks_for(ntc_max, 64), blocks_for(Hmax, 4 * kSegRows), n),
                       dim3(256), 0, s, d_args);
}

void launch_init_jobs(const Job *d_jobs, int njobs, int Hmax, int, hipStream_t s)
{
    hipLaunchKernelGGL(init_jobs_kernel, dim3(Hmax + 1, njobs), dim3(256), 0, s, d_jobs);
}

void launch_seg_finish(const SegFinish *d_args, int n, int ntc_max, int Hmax, hipStream_t s)
{
    hipLaunchKernelGGL(seg_finish_kernel, dim3(blocks_for(ntc_max, 64), blocks_for(Hmax, 4 * kSegRows), n),
                       dim3(256), 0, s, d_args);
}

void launch_energy(const Job *d_jobs, int njobs, int Hmax, int Wmax, hipStream_t s)
{
    hipLaunchKernelGGL(energy_kernel, dim3(blocks_for(tiles_across(Wmax), 64), blocks_for(Hmax, 16), njobs),
                       dim3(256), 0, s, d_jobs);
}

int DpGeom::cover(int W) const
{
    if (banded && R > 0) return W + chunk_waves() * C() + HB;
    if (banded) return waves(W) * C() + HB;
    const int t = (W + Q - 1) / Q;
    return ((t + 63) / 64) * 64 * Q;
}

int DpGeom::threads(int Wmax) const
{
    if (banded && R > 0) return 64 * chunk_waves();
    if (banded) return 64 * waves(Wmax);
    const int t = (Wmax + Q - 1) / Q;
    return ((t + 63) / 64) * 64;
}

// Banded variants (Q columns per lane, HB halo columns = rows per band, PF
// rows of key prefetch); for each (Q, HB) the first listed PF is the default.
const DpGeom kDpVariants[] = {{2, 8, 1, 8, 0},   {2, 8, 1, 16, 0},  {4, 8, 1, 8, 0},   {4, 8, 1, 16, 0},
                              {4, 16, 1, 8, 0},  {4, 16, 1, 16, 0}, {8, 16, 1, 4, 0},  {8, 16, 1, 8, 0},
                              {8, 16, 1, 16, 0}, {8, 32, 1, 4, 0},  {8, 32, 1, 8, 0},  {16, 32, 1, 2, 0},
                              {16, 32, 1, 4, 0}, {16, 32, 1, 8, 0}, {16, 64, 1, 2, 0}, {16, 64, 1, 4, 0}};
const int kNumDpVariants = (int)(sizeof(kDpVariants) / sizeof(kDpVariants[0]));

// Chunked variants (column-split DP, one launch per R rows).
const DpGeom kDpChunked[] = {
    {4, 16, 1, 8, 0, 256, 384},  {4, 16, 1, 8, 0, 384, 256},  {4, 16, 1, 8, 0, 320, 384}, {4, 16, 1, 8, 0, 192, 512},
    {4, 16, 1, 8, 0, 128, 640},  {4, 16, 1, 8, 0, 512, 768},  {4, 16, 1, 8, 0, 128, 768}, {4, 16, 1, 8, 0, 128, 1024},
    {4, 16, 1, 8, 0, 192, 896},  {4, 16, 1, 8, 0, 256, 768},  {4, 16, 1, 8, 0, 256, 1024}, {4, 16, 1, 8, 0, 320, 640},
    {4, 16, 1, 8, 0, 384, 128},  {4, 16, 1, 8, 0, 352, 192},  {4, 16, 1, 8, 0, 288, 320},
    {2, 8, 1, 16, 0, 128, 640},  {2, 8, 1, 16, 0, 64, 768},   {4, 8, 1, 8, 0, 128, 704},
    {2, 8, 1, 16, 0, 192, 64},   {2, 8, 1, 16, 0, 160, 128},  {2, 8, 1, 16, 0, 128, 192},
    {2, 8, 1, 16, 0, 208, 32},   {2, 8, 1, 16, 0, 216, 16},
    {4, 16, 1, 16, 0, 256, 384}, {4, 16, 1, 16, 0, 320, 384}, {4, 16, 1, 16, 0, 192, 512}};
const int kNumDpChunked = (int)(sizeof(kDpChunked) / sizeof(kDpChunked[0]));

bool dp_geom_fits(const DpGeom &g, int Wmax)
{
    if (!g.banded) return true;
    if (g.R > 0)  // the instantiated dp_chunk_kernel variants
        return ((g.Q == 4 && g.HB == 16 && (g.PF == 8 || g.PF == 16)) ||
                (g.Q == 2 && g.HB == 8 && g.PF == 16) || (g.Q == 4 && g.HB == 8 && g.PF == 8)) &&
               g.C() > 0 && g.P > 0 && g.P % g.Q == 0 && g.R % g.Q == 0 && g.R >= g.HB &&
               g.threads(Wmax) <= dp_max_threads(g.Q, g.PF) && (size_t)2 * g.chunk_waves() * g.C() * 4 <= 65536;
    return g.C() > 0 && g.threads(Wmax) <= dp_max_threads(g.Q, g.PF) && (size_t)2 * (g.cover(Wmax) + 64) * 4 <= 65536;
}

DpGeom dp_geom(int Wmax)
{
    // defaults (the autotuner may replace them): up to 448 columns, one
    // workgroup of four wavefronts; wider, the column-split DP (4,16,8) with
    // 256 rows by 384 columns per workgroup, which is faster than every
    // single-workgroup variant at any number of concurrent 1080- or 2160-row
    // buffers; beyond 8960 columns the row-synchronous kernel
    if (Wmax <= 448) return DpGeom{2, 8, 1, 8, 0};
    if (Wmax <= 8960) {
        DpGeom g{4, 16, 1, 8, 1};
        g.R = 256;
        g.P = 384;
        return g;
    }
    return DpGeom{32, 0, 0, 2, 0};
}

size_t g_dp_lds_cap = 65536;  // LDS of one compute unit as a workgroup may request it

void launch_dp(const Job *d_jobs, int njobs, const DpGeom &g, int Wmax, int Hmax, hipStream_t s)
{
    if (g.banded && g.R > 0) {
        const int ngx = g.groups(Wmax);
        // a job's workgroups on one XCD once every XCD has a job (with fewer
        // jobs, spreading them over all XCDs measured faster)
        const int xl = njobs >= 8 ? 1 : 0;
        const dim3 grid(xl ? ngx * ((njobs + 7) / 8) * 8 : ngx * njobs), block(g.threads(Wmax));
        size_t lds = (size_t)2 * g.chunk_waves() * g.C() * sizeof(uint32_t);
        if (g.EX && lds < g_dp_lds_cap) lds = g_dp_lds_cap;
#define SCPL_DPC_CASE(q, hb, pf)                                                                          \
    if (g.Q == q && g.HB == hb && g.PF == pf) {                                                           \
        for (int r0 = 0; r0 < Hmax; r0 += g.R)                                                            \
            hipLaunchKernelGGL((dp_chunk_kernel<q, hb, pf>), grid, block, lds, s, d_jobs, njobs, ngx, xl, r0,  \
                               g.R, g.P);                                                                 \
        return;                                                                                           \
    }
        SCPL_DPC_CASE(4, 16, 8)
        SCPL_DPC_CASE(4, 16, 16)
        SCPL_DPC_CASE(2, 8, 16)
        SCPL_DPC_CASE(4, 8, 8)
#undef SCPL_DPC_CASE
        return;
    }
    const dim3 grid(njobs), block(g.threads(Wmax));
    // two ping-pong rows of keys: the widest job's key row less its left pad
    size_t lds = g.banded ? (size_t)2 * (g.cover(Wmax) + 64) * sizeof(uint32_t) : 0;
    if (g.EX && lds < g_dp_lds_cap) lds = g_dp_lds_cap;
    if (!g.banded) {
        hipLaunchKernelGGL(dp_kernel<32>, grid, block, lds, s, d_jobs);
        return;
    }
#define SCPL_DP_CASE(q, hb, pf)                                                             \
    if (g.Q == q && g.HB == hb && g.PF == pf) {                                             \
        hipLaunchKernelGGL((dp_band_kernel<q, hb, pf>), grid, block, lds, s, d_jobs);    \
        return;                                                                             \
    }
    SCPL_DP_CASE(2, 8, 8)
    SCPL_DP_CASE(2, 8, 16)
    SCPL_DP_CASE(4, 8, 8)
    SCPL_DP_CASE(4, 8, 16)
    SCPL_DP_CASE(4, 16, 8)
    SCPL_DP_CASE(4, 16, 16)
    SCPL_DP_CASE(8, 16, 4)
    SCPL_DP_CASE(8, 16, 8)
    SCPL_DP_CASE(8, 16, 16)
    SCPL_DP_CASE(8, 32, 4)
    SCPL_DP_CASE(8, 32, 8)
    SCPL_DP_CASE(16, 32, 2)
    SCPL_DP_CASE(16, 32, 4)
    SCPL_DP_CASE(16, 32, 8)
    SCPL_DP_CASE(16, 64, 2)
    SCPL_DP_CASE(16, 64, 4)
#undef SCPL_DP_CASE
    hipLaunchKernelGGL(dp_kernel<32>, grid, block, 0, s, d_jobs);  // unreachable for valid geometries
}

// Deterministic pseudo-random key rows for the autotuner (xorshift of the
// position; values 0..7650).
__global__ void tune_fill_kernel(uint16_t *K, int H, int W, int Kp, int KL)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)H * W) return;
    const int i = (int)(p / W), j = (int)(p - (int64_t)i * W);
    uint32_t x = (uint32_t)p * 2654435761u + 12345u;
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    K[(size_t)i * Kp + KL + j] = (uint16_t)((x % 7651u) << 2);
}

void launch_tune_fill(uint16_t *K, int H, int W, int Kp, int KL, hipStream_t s)
{
    hipLaunchKernelGGL(tune_fill_kernel, dim3(blocks_for((int64_t)H * W, 256)), dim3(256), 0, s, K, H, W, Kp, KL);
}

template <int COLS>
static void launch_borg_v(const Job *d_jobs, int njobs, int nbmax, int Bmax, int Wmax, hipStream_t s)
{
    const size_t lds = (size_t)Bmax * (COLS + 2 * Bmax + 8);
    hipLaunchKernelGGL((borg_kernel<COLS>), dim3(blocks_for(Wmax, COLS), nbmax, njobs), dim3(COLS), lds, s, d_jobs);
}

void launch_borg(const Job *d_jobs, int njobs, int nbmax, int Bmax, int Wmax, int variant, hipStream_t s)
{
    if (variant == 1) launch_borg_v<128>(d_jobs, njobs, nbmax, Bmax, Wmax, s);
    else if (variant == 2) launch_borg_v<512>(d_jobs, njobs, nbmax, Bmax, Wmax, s);
    else launch_borg_v<kBorgCols>(d_jobs, njobs, nbmax, Bmax, Wmax, s);
}

void launch_labels(const Job *d_jobs, int njobs, int Wmax, hipStream_t s)
{
    hipLaunchKernelGGL(labels_kernel, dim3(blocks_for(Wmax, 256), njobs), dim3(256), 0, s, d_jobs);
}

size_t select_lds_bytes(size_t lds_cap) { return lds_cap; }

void set_kernel_attributes(size_t lds_cap)
{
    g_dp_lds_cap = lds_cap;
    const void *dps[] = {
        reinterpret_cast<const void *>(&dp_kernel<32>),          reinterpret_cast<const void *>(&dp_band_kernel<2, 8, 8>),
        reinterpret_cast<const void *>(&dp_band_kernel<2, 8, 16>), reinterpret_cast<const void *>(&dp_band_kernel<4, 8, 8>),
        reinterpret_cast<const void *>(&dp_band_kernel<4, 8, 16>), reinterpret_cast<const void *>(&dp_band_kernel<4, 16, 8>),
        reinterpret_cast<const void *>(&dp_band_kernel<4, 16, 16>), reinterpret_cast<const void *>(&dp_band_kernel<8, 16, 4>),
        reinterpret_cast<const void *>(&dp_band_kernel<8, 16, 8>), reinterpret_cast<const void *>(&dp_band_kernel<8, 32, 4>),
        reinterpret_cast<const void *>(&dp_band_kernel<16, 32, 2>), reinterpret_cast<const void *>(&dp_band_kernel<16, 64, 2>),
        reinterpret_cast<const void *>(&dp_band_kernel<8, 16, 16>), reinterpret_cast<const void *>(&dp_band_kernel<8, 32, 8>),
        reinterpret_cast<const void *>(&dp_band_kernel<16, 32, 4>), reinterpret_cast<const void *>(&dp_band_kernel<16, 32, 8>),
        reinterpret_cast<const void *>(&dp_band_kernel<16, 64, 4>), reinterpret_cast<const void *>(&dp_chunk_kernel<4, 16, 8>),
        reinterpret_cast<const void *>(&dp_chunk_kernel<2, 8, 16>), reinterpret_cast<const void *>(&dp_chunk_kernel<4, 8, 8>),
        reinterpret_cast<const void *>(&dp_chunk_kernel<4, 16, 16>)};
    for (const void *f : dps) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&select_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&band_update_kernel<8>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)band_update_lds(8));
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&band_update_kernel<16>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)band_update_lds(16));
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&persist_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)persist_lds_bytes());
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&persist_kernel<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)persist_lds_bytes());
}

void launch_select(const Job *d_jobs, int njobs, int use_lab_array, size_t lds_cap, hipStream_t s)
{
    hipLaunchKernelGGL(select_kernel, dim3(njobs), dim3(1024), lds_cap, s, d_jobs, (int)lds_cap, use_lab_array);
}

void launch_jump_only(const Job *d_jobs, int njobs, hipStream_t s)
{
    hipLaunchKernelGGL(jump_kernel, dim3(njobs), dim3(256), 0, s, d_jobs);
}

bool band_update_fits(int kmax, int Bmax) { return Bmax == kFuseB && kmax <= kUpdSeams; }

void launch_band_update(const Job *d_jobs, int njobs, int nbmax, int variant, hipStream_t s)
{
    if (variant == 2)
        hipLaunchKernelGGL(band_update_kernel<16>, dim3(nbmax, njobs), dim3(1024), band_update_lds(16), s, d_jobs);
    else
        hipLaunchKernelGGL(band_update_kernel<8>, dim3(nbmax, njobs), dim3(512), band_update_lds(8), s, d_jobs);
}

void launch_fill(const Job *d_jobs, int njobs, int kmax, int nbmax, int Bmax, hipStream_t s)
{
    const int gx = kmax < 1024 ? kmax : 1024;
    const size_t lds = (size_t)Bmax * (2 * Bmax + 8);
    hipLaunchKernelGGL(fill_kernel, dim3(gx, nbmax, njobs), dim3(64), lds, s, d_jobs);
}

const int kUpdateVariants[][2] = {{4, 2048}, {2, 2048}, {8, 2048}, {4, 1024}, {8, 1024}, {1, 2048}, {2, 1024}};
const int kNumUpdateVariants = (int)(sizeof(kUpdateVariants) / sizeof(kUpdateVariants[0]));

template <int ROWS, int SPAN>
static void launch_update_v(const Job *d_jobs, int njobs, int Hmax, hipStream_t s)
{
    hipLaunchKernelGGL((update_kernel<ROWS, SPAN>), dim3(blocks_for(Hmax, ROWS), njobs), dim3(64 * ROWS), 0, s,
                       d_jobs);
}

void launch_update(const Job *d_jobs, int njobs, int Hmax, int, int variant, hipStream_t s)
{
    switch (variant) {
    case 1: launch_update_v<2, 2048>(d_jobs, njobs, Hmax, s); break;
    case 2: launch_update_v<8, 2048>(d_jobs, njobs, Hmax, s); break;
    case 3: launch_update_v<4, 1024>(d_jobs, njobs, Hmax, s); break;
    case 4: launch_update_v<8, 1024>(d_jobs, njobs, Hmax, s); break;
    case 5: launch_update_v<1, 2048>(d_jobs, njobs, Hmax, s); break;
    case 6: launch_update_v<2, 1024>(d_jobs, njobs, Hmax, s); break;
    default: launch_update_v<4, 2048>(d_jobs, njobs, Hmax, s); break;
    }
}

void launch_refresh(const Job *d_jobs, int njobs, int, int Hmax, int variant, hipStream_t s)
{
    const dim3 g(blocks_for(Hmax, kRefreshRows), njobs);
    // variant 0: 1024 threads per block when the launch has few blocks, else 256
    const bool wide = variant == 2 || (variant == 0 && (int64_t)g.x * njobs < 2 * 256);
    if (wide) hipLaunchKernelGGL(refresh_kernel<1024>, g, dim3(1024), 0, s, d_jobs);
    else hipLaunchKernelGGL(refresh_kernel<256>, g, dim3(256), 0, s, d_jobs);
}

// frames staged per pass of the gather variants (0: the streamed kernel)
constexpr int kGatherFrames[] = {1, 2, 4, 8, 0};
const int kNumGatherVariants = (int)(sizeof(kGatherFrames) / sizeof(kGatherFrames[0]));

static void launch_gather_stream(const Job *d_jobs, int njobs, int Hmax, int inb_max, int outb_max, int wmax,
                                 hipStream_t s)
{
    const size_t ip = ((size_t)inb_max + 15) & ~(size_t)15;
    const size_t lds = std::min(kGatherLds, 2 * ip + 2 * (size_t)outb_max + (((size_t)2 * wmax + 15) & ~(size_t)15));
    if (inb_max <= 128 * 4 * 16)
        hipLaunchKernelGGL((gather_stream_kernel<4, 2>), dim3(Hmax, njobs), dim3(256), lds, s, d_jobs, (int)lds);
    else
        hipLaunchKernelGGL((gather_stream_kernel<8, 2>), dim3(Hmax, njobs), dim3(256), lds, s, d_jobs, (int)lds);
}

template <int FPB>
static void launch_gather_v(const Job *d_jobs, int njobs, int Hmax, int inb_max, int outb_max, hipStream_t s)
{
    const size_t ip = ((size_t)inb_max + 15) & ~(size_t)15;
    size_t lds = (size_t)FPB * ip + 2 * (size_t)outb_max;
    if (lds > kGatherLds) lds = 0;  // every row of the launch gathers directly
    hipLaunchKernelGGL((gather_kernel<FPB>), dim3(Hmax, njobs), dim3(256), lds, s, d_jobs, (int)lds);
}

void launch_gather(const Job *d_jobs, int njobs, int Hmax, int inb_max, int outb_max, int wmax, int variant,
                   hipStream_t s)
{
    int v = std::min(std::max(variant, 0), kNumGatherVariants - 1);
    if (kGatherFrames[v] == 0) {
        launch_gather_stream(d_jobs, njobs, Hmax, inb_max, outb_max, wmax, s);
        return;
    }
    // fewer frames per pass when the variant's rows do not fit the LDS
    const size_t ip = ((size_t)inb_max + 15) & ~(size_t)15;
    while (v > 0 && (size_t)kGatherFrames[v] * ip + 2 * (size_t)outb_max > kGatherLds) --v;
    switch (kGatherFrames[v]) {
    case 2: launch_gather_v<2>(d_jobs, njobs, Hmax, inb_max, outb_max, s); break;
    case 4: launch_gather_v<4>(d_jobs, njobs, Hmax, inb_max, outb_max, s); break;
    case 8: launch_gather_v<8>(d_jobs, njobs, Hmax, inb_max, outb_max, s); break;
    default: launch_gather_v<1>(d_jobs, njobs, Hmax, inb_max, outb_max, s); break;
    }
}

size_t persist_lds_bytes()
{
    // the selection's keys of a 1920-column frame (30 KB) and four rows of
    // band origins beside them; the other stages need less
    size_t b = (size_t)2 * 1920 * 8 + 4 * (1920 + 8);
    b = std::max(b, band_update_lds(kPersistThreads / 64));
    b = std::max(b, sizeof(RefreshLds));
    b = std::max(b, (size_t)2 * 4 * (64 * 4 - 2 * 16) * sizeof(uint32_t));  // DP (4, 16, 8), four wavefronts
    b = std::max(b, (size_t)kFuseB * (kPersistThreads + 2 * kFuseB + 8));  // band origins
    return (b + 15) & ~(size_t)15;
}

int persist_blocks_per_cu()
{
    int n = 0, m = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(&persist_kernel<true>),
                                                     kPersistThreads, persist_lds_bytes()) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, reinterpret_cast<const void *>(&persist_kernel<false>),
                                                     kPersistThreads, persist_lds_bytes()) != hipSuccess)
        return 0;
    return std::min(n, m);
}

void launch_persist_clear(const PArgs &a, hipStream_t s)
{
    const int n = std::max(a.nring * (a.cap_mask + 1), std::max(a.njobs, a.nring));
    hipLaunchKernelGGL(persist_clear_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
}

int probe_xcc(int n, int *h_out)
{
    int *d = nullptr;
    if (hipMalloc(&d, sizeof(int) * (size_t)n) != hipSuccess) return -1;
    hipLaunchKernelGGL(xcc_probe_kernel, dim3(n), dim3(64), 0, nullptr, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(h_out, d, sizeof(int) * (size_t)n, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    return e == hipSuccess ? 0 : -1;
}

void launch_persist_seed(const PArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(persist_seed_kernel, dim3(1), dim3(64), 0, s, a);
}

void launch_persist(const PArgs &a, int grid, bool local, hipStream_t s)
{
    if (local) hipLaunchKernelGGL(persist_kernel<true>, dim3(grid), dim3(kPersistThreads), (size_t)a.lds_bytes, s, a);
    else hipLaunchKernelGGL(persist_kernel<false>, dim3(grid), dim3(kPersistThreads), (size_t)a.lds_bytes, s, a);
}

void launch_u_to_keys(const int32_t *src, uint16_t *dst, int H, int W, int pitch, int32_t *bad, hipStream_t s)
{
    hipLaunchKernelGGL(u_to_keys_kernel, dim3(blocks_for((int64_t)H * W, 256)), dim3(256), 0, s, src, dst, H, W,
                       pitch, bad);
}

void launch_keys_to_u(const uint16_t *src, int32_t *dst, int H, int W, int pitch, hipStream_t s)
{
    hipLaunchKernelGGL(keys_to_u_kernel, dim3(blocks_for((int64_t)H * W, 256)), dim3(256), 0, s, src, dst, H, W,
                       pitch);
}

void launch_transpose(const uint8_t *src, int N, int H, int W, int C, uint8_t *dst, hipStream_t s)
{
    const dim3 g(blocks_for(W, 32), blocks_for(H, 32), N);
    if (C == 3) hipLaunchKernelGGL(transpose_kernel<3>, g, dim3(256), 0, s, src, H, W, dst);
    else hipLaunchKernelGGL(transpose_kernel<1>, g, dim3(256), 0, s, src, H, W, dst);
}

void launch_transpose16(const uint16_t *src, int N, int H, int W, uint16_t *dst, hipStream_t s)
{
    const dim3 g(blocks_for(W, 32), blocks_for(H, 32), N);
    hipLaunchKernelGGL(transpose_kernel<2>, g, dim3(256), 0, s, reinterpret_cast<const uint8_t *>(src), H, W,
                       reinterpret_cast<uint8_t *>(dst));
}

void launch_compact_frame(const uint8_t *in, int H, int W, int C, const int32_t *seams, int kk, uint8_t *out,
                          hipStream_t s)
{
    hipLaunchKernelGGL(compact_frame_kernel, dim3(H), dim3(256), 0, s, in, H, W, C, seams, kk, out);
}

void launch_seams_out(const int16_t *src, int pitch, int32_t *dst, int kk, int H, hipStream_t s)
{
    hipLaunchKernelGGL(seams_out_kernel, dim3(blocks_for((int64_t)kk * H, 256)), dim3(256), 0, s, src, pitch, dst,
                       kk, H);
}

void launch_dir_out(const uint8_t *codes, int pitch, int8_t *dst, int H, int W, hipStream_t s)
{
    hipLaunchKernelGGL(dir_out_kernel, dim3(blocks_for((int64_t)H * W, 256)), dim3(256), 0, s, codes, pitch, dst, H,
                       W);
}

void launch_dir_in(const int8_t *src, uint8_t *codes, int pitch, int H, int W, hipStream_t s)
{
    hipLaunchKernelGGL(dir_in_kernel, dim3(blocks_for((int64_t)H * W, 256)), dim3(256), 0, s, src, codes, pitch, H,
                       W);
}

}  // namespace scpl
