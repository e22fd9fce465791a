// Warm-start network: training and inference kernels (FP32 storage and
// arithmetic; weight-gradient sums in FP64 so that they do not depend on the
// batch size's rounding).
//
//   layer  in -> out  3x3 kernel, dilation  activation
//     1     2 ->  32        1                ReLU
//     2    32 ->  32        2                ReLU
//     3    32 ->  32        4                ReLU
//     4    32 ->   2        8                none
// Zero padding equal to the dilation keeps the image size.  Tensors are NCHW.
// Parameters are one flat array: per layer W[out][in][3][3] then b[out].
//
// The network's input is the pair of marginals as densities averaged over a
// 32 x 32 partition of the square; its output is the pair of dual potentials in
// normalised coordinates, which inference interpolates back to the problem's
// pixels and scales to pixel cost units.
#include "internal.h"

namespace otip {

namespace {

constexpr int kCB = 256;  // threads per block

struct LayerSpec {
    int cin, cout, dil, relu;
};
constexpr LayerSpec kLayers[4] = {{2, 32, 1, 1}, {32, 32, 2, 1}, {32, 32, 4, 1}, {32, 2, 8, 0}};

__host__ __device__ constexpr int64_t layer_params(int l) {
    return (int64_t)kLayers[l].cout * kLayers[l].cin * 9 + kLayers[l].cout;
}

// out[n][o][y][x] = b[o] + sum_{c,ky,kx} W[o][c][ky][kx] in[n][c][y+(ky-1)d][x+(kx-1)d]
// grid (pixel blocks, cout, batch)
__global__ __launch_bounds__(kCB) void conv_fwd(int cin, int cout, int H, int W, int dil,
                                                const float *__restrict__ in,
                                                const float *__restrict__ wt,
                                                const float *__restrict__ bias,
                                                float *__restrict__ out, int relu) {
    __shared__ float ws[32 * 9];
    const int o = blockIdx.y, n = blockIdx.z;
    for (int t = threadIdx.x; t < cin * 9; t += kCB) ws[t] = wt[(size_t)o * cin * 9 + t];
    __syncthreads();
    const int p = blockIdx.x * kCB + threadIdx.x;
    if (p >= H * W) return;
    const int y = p / W, x = p % W;
    float acc = bias[o];
    for (int c = 0; c < cin; ++c) {
        const float *src = in + ((size_t)n * cin + c) * H * W;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int yy = y + (ky - 1) * dil;
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int xx = x + (kx - 1) * dil;
                if (xx < 0 || xx >= W) continue;
                acc = fmaf(ws[c * 9 + ky * 3 + kx], src[yy * W + xx], acc);
            }
        }
    }
    if (relu) acc = fmaxf(acc, 0.0f);
    out[((size_t)n * cout + o) * H * W + p] = acc;
}

// gin[n][c][y][x] = sum_{o,ky,kx} W[o][c][ky][kx] g[n][o][y-(ky-1)d][x-(kx-1)d],
// then times [act > 0] (act = the ReLU output that was this layer's input)
// grid (pixel blocks, cin, batch)
__global__ __launch_bounds__(kCB) void conv_bwd_data(int cin, int cout, int H, int W, int dil,
                                                     const float *__restrict__ g,
                                                     const float *__restrict__ wt,
                                                     const float *__restrict__ act,
                                                     float *__restrict__ gin) {
    __shared__ float ws[32 * 9];
    const int c = blockIdx.y, n = blockIdx.z;
    for (int t = threadIdx.x; t < cout * 9; t += kCB) {
        const int o = t / 9, k = t % 9;
        ws[t] = wt[((size_t)o * cin + c) * 9 + k];
    }
    __syncthreads();
    const int p = blockIdx.x * kCB + threadIdx.x;
    if (p >= H * W) return;
    const int y = p / W, x = p % W;
    float acc = 0.0f;
    for (int o = 0; o < cout; ++o) {
        const float *src = g + ((size_t)n * cout + o) * H * W;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int yy = y - (ky - 1) * dil;
            if (yy < 0 || yy >= H) continue;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int xx = x - (kx - 1) * dil;
                if (xx < 0 || xx >= W) continue;
                acc = fmaf(ws[o * 9 + ky * 3 + kx], src[yy * W + xx], acc);
            }
        }
    }
    const size_t q = ((size_t)n * cin + c) * H * W + p;
    gin[q] = act[q] > 0.0f ? acc : 0.0f;
}

// gW[o][c][ky][kx] = sum_{n,y,x} g[n][o][y][x] in[n][c][y+(ky-1)d][x+(kx-1)d];
// block (c, o); c == cin gives gb[o] = sum g[n][o][y][x].  Fixed-order sums.
__global__ __launch_bounds__(kCB) void conv_bwd_weights(int N, int cin, int cout, int H, int W,
                                                        int dil, const float *__restrict__ g,
                                                        const float *__restrict__ in,
                                                        float *__restrict__ gw,
                                                        float *__restrict__ gb) {
    __shared__ double red[9][kCB / 64];
    const int c = blockIdx.x, o = blockIdx.y;
    const bool bias = c == cin;
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    const int HW = H * W;
    const int64_t total = (int64_t)N * HW;
    for (int64_t e = threadIdx.x; e < total; e += kCB) {
        const int n = (int)(e / HW), p = (int)(e % HW);
        const float gv = g[((size_t)n * cout + o) * HW + p];
        if (bias) {
            acc[0] += (double)gv;
            continue;
        }
        const int y = p / W, x = p % W;
        const float *src = in + ((size_t)n * cin + c) * HW;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            const int yy = y + (ky - 1) * dil;
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int xx = x + (kx - 1) * dil;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    acc[ky * 3 + kx] = fma((double)gv, (double)src[yy * W + xx], acc[ky * 3 + kx]);
            }
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) red[k][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double v = 0.0;
        for (int q = 0; q < kCB / 64; ++q) v += red[threadIdx.x][q];
        if (bias) {
            if (threadIdx.x == 0) gb[o] = (float)v;
        } else {
            gw[((size_t)o * cin + c) * 9 + threadIdx.x] = (float)v;
        }
    }
}

// g = 2 (out - target) / count; per-block partial sums of (out - target)^2
__global__ __launch_bounds__(kCB) void mse_grad(int64_t count, const float *__restrict__ out,
                                                const float *__restrict__ target,
                                                float *__restrict__ g, double *part) {
    __shared__ double lds[16];
    double s = 0.0;
    const float scale = 2.0f / (float)count;
    for (int64_t e = (int64_t)blockIdx.x * kCB + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * kCB) {
        const float d = out[e] - target[e];
        g[e] = scale * d;
        s = fma((double)d, (double)d, s);
    }
    s = block_sum(s, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// omb = 1 - beta, formed in FP64 by the caller (1 - 0.999f loses 4 digits)
__global__ void adam_update(int64_t count, float *__restrict__ w, float *__restrict__ m,
                            float *__restrict__ v, const float *__restrict__ g, float lr,
                            float b1, float b2, float omb1, float omb2, float c1, float c2,
                            float eps) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float ge = g[e];
    const float me = b1 * m[e] + omb1 * ge;
    const float ve = b2 * v[e] + omb2 * ge * ge;
    m[e] = me;
    v[e] = ve;
    w[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
}

// network input from one problem: each marginal times side^2 (a density),
// averaged over the cells of the grid x grid partition of the square
__global__ void ws_input(int side, int grid, const double *__restrict__ a,
                         const double *__restrict__ b, float *__restrict__ x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * grid * grid) return;
    const int ch = t / (grid * grid), ty = (t / grid) % grid, tx = t % grid;
    const double *h = ch == 0 ? a : b;
    // source pixels overlapping [ty, ty+1) / grid
    const int u0 = (int)floor((double)ty * side / grid);
    const int u1 = min(side, (int)ceil((double)(ty + 1) * side / grid));
    const int v0 = (int)floor((double)tx * side / grid);
    const int v1 = min(side, (int)ceil((double)(tx + 1) * side / grid));
    const double g0y = (double)ty / grid, g1y = (double)(ty + 1) / grid;
    const double g0x = (double)tx / grid, g1x = (double)(tx + 1) / grid;
    double acc = 0.0;
    for (int u = u0; u < u1; ++u) {
        const double oy = fmax(0.0, fmin(g1y, (double)(u + 1) / side) - fmax(g0y, (double)u / side));
        for (int v = v0; v < v1; ++v) {
            const double ox =
                fmax(0.0, fmin(g1x, (double)(v + 1) / side) - fmax(g0x, (double)v / side));
            acc += h[u * side + v] * (oy * grid) * (ox * grid);
        }
    }
    x[t] = (float)(acc * side * side);
}

// duals at the problem's pixel centres: bilinear in the grid x grid output,
// clamped at the border, times side^2
__global__ void ws_output(int side, int grid, const float *__restrict__ out, double *y0,
                          double *z0) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * side * side) return;
    const int ch = t / (side * side), r = (t / side) % side, c = t % side;
    auto coord = [&](int u) {
        double s = ((double)u + 0.5) * grid / side - 0.5;
        return fmin(fmax(s, 0.0), (double)(grid - 1));
    };
    const double tr = coord(r), tc = coord(c);
    const int r0 = (int)floor(tr), c0 = (int)floor(tc);
    const int r1 = min(r0 + 1, grid - 1), c1 = min(c0 + 1, grid - 1);
    const double fr = tr - r0, fc = tc - c0;
    const float *P = out + (size_t)ch * grid * grid;
    const double top = (double)P[r0 * grid + c0] * (1.0 - fc) + (double)P[r0 * grid + c1] * fc;
    const double bot = (double)P[r1 * grid + c0] * (1.0 - fc) + (double)P[r1 * grid + c1] * fc;
    const double v = (top * (1.0 - fr) + bot * fr) * side * side;
    (ch == 0 ? y0 : z0)[r * side + c] = v;
}

}  // namespace

int64_t WarmNet::param_count() {
    int64_t s = 0;
    for (int l = 0; l < 4; ++l) s += layer_params(l);
    return s;
}

void WarmNet::forward(hipStream_t st, const float *theta, int N, int H, int W, const float *x,
                      float *out) {
    const size_t hw = (size_t)H * W;
    float *act[3] = {a_[0].need((size_t)N * 32 * hw), a_[1].need((size_t)N * 32 * hw),
                     a_[2].need((size_t)N * 32 * hw)};
    const float *in = x;
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
        const LayerSpec L = kLayers[l];
        float *dst = l < 3 ? act[l] : out;
        dim3 grid(grid_for((int64_t)hw, kCB), L.cout, N);
        hipLaunchKernelGGL(conv_fwd, grid, dim3(kCB), 0, st, L.cin, L.cout, H, W, L.dil, in,
                           theta + off, theta + off + (int64_t)L.cout * L.cin * 9, dst, L.relu);
        off += layer_params(l);
        in = dst;
    }
    OTIP_HIP(hipGetLastError());
}

double WarmNet::grad(hipStream_t st, const float *theta, int N, int H, int W, const float *x,
                     const float *target, float *g) {
    const size_t hw = (size_t)H * W;
    float *out = out_.need((size_t)N * 2 * hw);
    forward(st, theta, N, H, W, x, out);
    const int64_t cnt = (int64_t)N * 2 * hw;
    float *gcur = ga_.need((size_t)N * 32 * hw);
    float *gnext = gb_.need((size_t)N * 32 * hw);
    const int pb = (int)std::min<int64_t>(1024, grid_for(cnt, kCB));
    double *part = part_.need(pb);
    hipLaunchKernelGGL(mse_grad, dim3(pb), dim3(kCB), 0, st, cnt, out, target, gcur, part);
    int64_t offs[4], off = 0;
    for (int l = 0; l < 4; ++l) {
        offs[l] = off;
        off += layer_params(l);
    }
    for (int l = 3; l >= 0; --l) {
        const LayerSpec L = kLayers[l];
        const float *xin = l == 0 ? x : a_[l - 1].get();
        float *gw = g + offs[l];
        float *gbias = gw + (int64_t)L.cout * L.cin * 9;
        hipLaunchKernelGGL(conv_bwd_weights, dim3(L.cin + 1, L.cout), dim3(kCB), 0, st, N, L.cin,
                           L.cout, H, W, L.dil, gcur, xin, gw, gbias);
        if (l > 0) {
            dim3 grid(grid_for((int64_t)hw, kCB), L.cin, N);
            hipLaunchKernelGGL(conv_bwd_data, grid, dim3(kCB), 0, st, L.cin, L.cout, H, W, L.dil,
                               gcur, theta + offs[l], xin, gnext);
            std::swap(gcur, gnext);
        }
    }
    OTIP_HIP(hipGetLastError());
    std::vector<double> hp(pb);
    OTIP_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * pb, hipMemcpyDeviceToHost, st));
    OTIP_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double v : hp) s += v;
    return s / (double)cnt;
}

void WarmNet::adam(hipStream_t st, float *theta, float *m, float *v, const float *g, int step,
                   double lr, double b1, double b2, double eps) {
    const int64_t P = param_count();
    const float c1 = (float)(1.0 - std::pow(b1, step));
    const float c2 = (float)(1.0 - std::pow(b2, step));
    hipLaunchKernelGGL(adam_update, dim3(grid_for(P, 256)), dim3(256), 0, st, P, theta, m, v, g,
                       (float)lr, (float)b1, (float)b2, (float)(1.0 - b1), (float)(1.0 - b2), c1,
                       c2, (float)eps);
    OTIP_HIP(hipGetLastError());
}

void WarmNet::predict(hipStream_t st, const float *theta, int side, const double *a,
                      const double *b, double *y0, double *z0) {
    constexpr int G = 32;
    float *x = in_.need(2 * G * G);
    float *out = out_.need(2 * G * G);
    hipLaunchKernelGGL(ws_input, dim3(grid_for(2 * G * G, 256)), dim3(256), 0, st, side, G, a, b,
                       x);
    forward(st, theta, 1, G, G, x, out);
    hipLaunchKernelGGL(ws_output, dim3(grid_for(2 * (int64_t)side * side, 256)), dim3(256), 0, st,
                       side, G, out, y0, z0);
    OTIP_HIP(hipGetLastError());
}

}  // namespace otip
