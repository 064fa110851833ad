/*
 * FP64 oracle for the surrogate network: a plain multilayer perceptron
 * (ReLU on every hidden layer, or a sine on the first one, linear output),
 * its training loss and its gradients by ordinary back-propagation.
 *
 * First hidden layer: h = relu(z) when omega0 = 0, else h = sin(omega0 z)
 * (a sinusoidal layer of fixed frequency omega0, whose derivative is
 * omega0 cos(omega0 z)); z = W_0 x + b_0.  Every later hidden layer is ReLU.
 *
 * TEST INFRASTRUCTURE ONLY (see cvib_oracle.c).  Shares no code with the HIP
 * kernels.  Layer l maps d_l inputs to d_{l+1} outputs: y = W_l x + b_l with
 * W_l stored row-major as [d_{l+1}][d_l]; all layers' weights are concatenated
 * into one flat array in layer order, and likewise the biases.
 *
 * Loss (per batch of B samples, D outputs; the first D-1 outputs predict the
 * per-angle-bin radii, the last one is the feasibility logit):
 *   L = (1/B) sum_s [ (1/(D-1)) sum_k m_sk huber(out_sk - t_sk)
 *                     + bce_logits(out_s,D-1 ; f_s) ]
 *   m_sk = (t_sk > 0)   (a bin without a valid radius carries no radius loss)
 *   huber(e) = e^2/2 if |e| <= delta, else delta (|e| - delta/2)
 *   bce_logits(z; f) = max(z,0) - z f + log(1 + exp(-|z|))
 * The gradient w.r.t. the outputs is written by orc_mlp_loss.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int64_t total_hidden(const int32_t* dims, int32_t nl) {
    int64_t s = 0;
    for (int l = 1; l < nl; ++l) s += dims[l];
    return s;
}

/* Forward pass for one sample; h receives the post-ReLU hidden activations of
 * layers 1..nl-1 back to back (size total_hidden). */
static void forward1(const int32_t* dims, int32_t nl, const double* W, const double* b,
                     const double* x, double* h, double* out, double omega0) {
    const double* in = x;
    double* hp = h;
    int64_t ow = 0, ob = 0;
    for (int l = 0; l < nl; ++l) {
        int32_t di = dims[l], dout = dims[l + 1];
        double* dst = (l == nl - 1) ? out : hp;
        for (int32_t o = 0; o < dout; ++o) {
            double acc = b[ob + o];
            for (int32_t k = 0; k < di; ++k) acc += W[ow + (int64_t)o * di + k] * in[k];
            if (l == nl - 1) dst[o] = acc;
            else if (l == 0 && omega0 > 0.0) dst[o] = sin(omega0 * acc);
            else dst[o] = acc > 0.0 ? acc : 0.0;
        }
        ow += (int64_t)dout * di;
        ob += dout;
        if (l < nl - 1) {
            in = hp;
            hp += dout;
        }
    }
}

void orc_mlp_forward(const int32_t* dims, int32_t nl, const double* W, const double* b,
                     int64_t B, const double* x, double* out, double omega0) {
    int64_t H = total_hidden(dims, nl);
    double* h = (double*)malloc(sizeof(double) * (size_t)(H > 0 ? H : 1));
    for (int64_t s = 0; s < B; ++s)
        forward1(dims, nl, W, b, x + s * dims[0], h, out + s * dims[nl], omega0);
    free(h);
}

double orc_mlp_loss(const double* out, const double* tr, const double* tf, int64_t B,
                    int32_t D, double delta, double* grad) {
    double total = 0.0;
    const int32_t R = D - 1;
    for (int64_t s = 0; s < B; ++s) {
        double ls = 0.0;
        for (int32_t k = 0; k < R; ++k) {
            double t = tr[s * R + k];
            double g = 0.0;
            if (t > 0.0) {
                double e = out[s * D + k] - t;
                double ae = fabs(e);
                ls += (ae <= delta ? 0.5 * e * e : delta * (ae - 0.5 * delta)) / R;
                g = (ae <= delta ? e : (e > 0 ? delta : -delta)) / R;
            }
            if (grad) grad[s * D + k] = g / (double)B;
        }
        double z = out[s * D + R], f = tf[s];
        ls += (z > 0 ? z : 0.0) - z * f + log1p(exp(-fabs(z)));
        if (grad) grad[s * D + R] = (1.0 / (1.0 + exp(-z)) - f) / (double)B;
        total += ls;
    }
    return total / (double)B;
}

/* Gradients of sum_s sum_o gout[s][o] * out[s][o] with respect to W and b
 * (accumulated over the batch into gW, gb, which are overwritten). */
void orc_mlp_backward(const int32_t* dims, int32_t nl, const double* W, const double* b,
                      int64_t B, const double* x, const double* gout, double* gW, double* gb,
                      double omega0) {
    int64_t nW = 0, nb = 0, H = total_hidden(dims, nl);
    int32_t dmax = 0;
    for (int l = 0; l < nl; ++l) {
        nW += (int64_t)dims[l] * dims[l + 1];
        nb += dims[l + 1];
    }
    for (int l = 0; l <= nl; ++l) dmax = dims[l] > dmax ? dims[l] : dmax;
    memset(gW, 0, sizeof(double) * (size_t)nW);
    memset(gb, 0, sizeof(double) * (size_t)nb);
    double* h = (double*)malloc(sizeof(double) * (size_t)(H > 0 ? H : 1));
    double* out = (double*)malloc(sizeof(double) * (size_t)dims[nl]);
    double* delta = (double*)malloc(sizeof(double) * (size_t)dmax);
    double* prev = (double*)malloc(sizeof(double) * (size_t)dmax);
    int64_t* offW = (int64_t*)malloc(sizeof(int64_t) * (size_t)nl);
    int64_t* offb = (int64_t*)malloc(sizeof(int64_t) * (size_t)nl);
    int64_t* offh = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nl + 1));
    int64_t aw = 0, ab = 0, ah = 0;
    for (int l = 0; l < nl; ++l) {
        offW[l] = aw;
        offb[l] = ab;
        aw += (int64_t)dims[l] * dims[l + 1];
        ab += dims[l + 1];
    }
    for (int l = 1; l < nl; ++l) {
        offh[l] = ah;
        ah += dims[l];
    }
    for (int64_t s = 0; s < B; ++s) {
        const double* xs = x + s * dims[0];
        forward1(dims, nl, W, b, xs, h, out, omega0);
        for (int32_t o = 0; o < dims[nl]; ++o) delta[o] = gout[s * dims[nl] + o];
        for (int l = nl - 1; l >= 0; --l) {
            int32_t di = dims[l], dout = dims[l + 1];
            const double* in = (l == 0) ? xs : h + offh[l];
            /* delta holds dLoss/d(pre-activation of layer l's output) */
            for (int32_t o = 0; o < dout; ++o) {
                gb[offb[l] + o] += delta[o];
                for (int32_t k = 0; k < di; ++k)
                    gW[offW[l] + (int64_t)o * di + k] += delta[o] * in[k];
            }
            if (l == 0) break;
            for (int32_t k = 0; k < di; ++k) {
                double acc = 0.0;
                for (int32_t o = 0; o < dout; ++o) acc += W[offW[l] + (int64_t)o * di + k] * delta[o];
                if (l == 1 && omega0 > 0.0) {
                    /* sine derivative at the first hidden layer: omega0 cos(omega0 z),
                     * z = W_0 x + b_0 recomputed */
                    double z = b[k];
                    for (int32_t c = 0; c < dims[0]; ++c) z += W[(int64_t)k * dims[0] + c] * xs[c];
                    prev[k] = acc * omega0 * cos(omega0 * z);
                } else {
                    /* ReLU derivative at the input of this layer (output of l-1) */
                    prev[k] = in[k] > 0.0 ? acc : 0.0;
                }
            }
            memcpy(delta, prev, sizeof(double) * (size_t)di);
        }
    }
    free(h); free(out); free(delta); free(prev); free(offW); free(offb); free(offh);
}

/* Gradient with respect to the input of one linear layer y = W x + b:
 * gin[s][k] = sum_o gout[s][o] W[o][k] (W row-major [dout][din]); the chain
 * rule's step from a layer's output gradient to its input. */
void orc_linear_input_grad(int32_t din, int32_t dout, const double* W, int64_t B, const double* gout,
                           double* gin) {
    for (int64_t s = 0; s < B; ++s)
        for (int32_t k = 0; k < din; ++k) {
            double acc = 0.0;
            for (int32_t o = 0; o < dout; ++o) acc += gout[s * dout + o] * W[(int64_t)o * din + k];
            gin[s * din + k] = acc;
        }
}
