// Exact piecewise-linear expansion of the one-input index network.
//
// With one input u the network y(u) = W3 act(W2 act(W1 u + b1) + b2) + b3 is
// piecewise linear: first-layer units switch at u = -b1_j / W1_j; between
// consecutive first-layer switches every second-layer pre-activation is
// linear in u and switches at most once.  Collecting all switch points gives
// the pieces; on each piece the output is slope * u + intercept, evaluated
// here in float64 from the trained float32 weights.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace symed {

namespace {

struct Net {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
    double mu, sc;  // network input x = (u - mu) * sc
};

inline bool passes(double z, int j) { return (j < kHidden / 2) ? (z > 0.0) : (z < 0.0); }

// first-layer unit j as a linear function of u at the point m
inline void layer1(const Net &n, int j, double m, double &a, double &b)
{
    const double w = (double)n.W1[j] * n.sc, c = (double)n.b1[j] - (double)n.W1[j] * n.sc * n.mu;
    if (passes(w * m + c, j)) { a = w; b = c; } else { a = 0.0; b = 0.0; }
}

// second-layer pre-activations A_k u + B_k, linear around the point m
void layer2(const Net &n, double m, std::vector<double> &A, std::vector<double> &B)
{
    const int H = kHidden;
    double a1[kHidden], c1[kHidden];
    for (int j = 0; j < H; ++j) layer1(n, j, m, a1[j], c1[j]);
    for (int k = 0; k < H; ++k) {
        double a = 0.0, b = n.b2[k];
        for (int j = 0; j < H; ++j) {
            a += (double)n.W2[k * H + j] * a1[j];
            b += (double)n.W2[k * H + j] * c1[j];
        }
        A[k] = a;
        B[k] = b;
    }
}

double direct(const Net &n, double u)
{
    const int H = kHidden;
    double h1[kHidden];
    for (int j = 0; j < H; ++j) {
        const double z = (double)n.W1[j] * ((u - n.mu) * n.sc) + n.b1[j];
        h1[j] = (j < H / 2) ? std::max(z, 0.0) : std::min(z, 0.0);
    }
    double y = n.b3[0];
    for (int k = 0; k < H; ++k) {
        double z = n.b2[k];
        for (int j = 0; j < H; ++j) z += (double)n.W2[k * H + j] * h1[j];
        y += (double)n.W3[k] * ((k < H / 2) ? std::max(z, 0.0) : std::min(z, 0.0));
    }
    return y;
}

}  // namespace

// params: float32 weights of the one-input network.  block: kPwFloats floats
// (header n, breakpoints, slopes, intercepts).  Returns the number of pieces,
// and in *max_dev the largest |expansion - network| over a test grid.
int expand_network(const float *params, float mu, float sc, std::vector<float> &block, double *max_dev)
{
    const int H = kHidden, F = 1;
    Net n;
    n.mu = mu;
    n.sc = sc;
    n.W1 = params;
    n.b1 = n.W1 + H * F;
    n.W2 = n.b1 + H;
    n.b2 = n.W2 + H * H;
    n.W3 = n.b2 + H;
    n.b3 = n.W3 + H;
    std::vector<double> br1;
    for (int j = 0; j < H; ++j)
        if (n.W1[j] != 0.0f) br1.push_back(n.mu - (double)n.b1[j] / ((double)n.W1[j] * n.sc));
    std::sort(br1.begin(), br1.end());
    br1.erase(std::unique(br1.begin(), br1.end()), br1.end());
    std::vector<double> brk = br1, A(H), B(H);
    // intervals between first-layer switches
    for (size_t i = 0; i <= br1.size(); ++i) {
        const double lo = (i == 0) ? -INFINITY : br1[i - 1];
        const double hi = (i == br1.size()) ? INFINITY : br1[i];
        double m;
        if (br1.empty()) m = 0.0;
        else if (i == 0) m = br1[0] - 1.0;
        else if (i == br1.size()) m = br1.back() + 1.0;
        else m = 0.5 * (lo + hi);
        layer2(n, m, A, B);
        for (int k = 0; k < H; ++k)
            if (A[k] != 0.0) {
                const double t = -B[k] / A[k];
                if (t > lo && t < hi) brk.push_back(t);
            }
    }
    std::sort(brk.begin(), brk.end());
    brk.erase(std::unique(brk.begin(), brk.end()), brk.end());
    const int pieces = (int)brk.size() + 1;
    block.assign(pw_floats(pieces), 0.0f);
    block[0] = (float)pieces;
    float *fb = block.data() + kPwHeader, *fs = block.data() + kPwHeader + pieces,
          *fi = block.data() + kPwHeader + 2 * pieces;
    for (int p = 0; p < pieces; ++p) {
        double m;
        if (brk.empty()) m = 0.0;
        else if (p == 0) m = brk[0] - 1.0;
        else if (p == pieces - 1) m = brk.back() + 1.0;
        else m = 0.5 * (brk[p - 1] + brk[p]);
        layer2(n, m, A, B);
        double s = 0.0, c = n.b3[0];
        for (int k = 0; k < H; ++k)
            if (passes(A[k] * m + B[k], k)) {
                s += (double)n.W3[k] * A[k];
                c += (double)n.W3[k] * B[k];
            }
        fs[p] = (float)s;
        fi[p] = (float)c;
        if (p < pieces - 1) fb[p] = (float)brk[p];
    }
    // check the expansion against the network on a grid of inputs
    double dev = 0.0;
    for (int q = 0; q <= 4096; ++q) {
        const double u = q / 4096.0;
        int lo = 0, hi = pieces - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((float)u < fb[mid]) hi = mid; else lo = mid + 1;
        }
        const double ye = (double)fs[lo] * u + fi[lo];
        dev = std::max(dev, std::fabs(ye - direct(n, u)));
    }
    *max_dev = dev;
    return pieces;
}

}  // namespace symed
