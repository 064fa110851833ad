"""Surrogate network kernels on the GPU: forward, loss, backward, Adam,
save / load and a short training run.

Two references: the FP64 oracle, given the same BF16-rounded weights, and a
plain PyTorch FP32 CPU emulation that rounds at the same points as the
kernels (hidden activations and back-propagated gradients to BF16).  Both
the ReLU first layer and the sinusoidal one (omega0 = 30) are checked.

Bars (norm-wise relative error):
- forward: 2e-2 against the oracle, 2e-3 against the emulation;
- gradients: 5e-2 against the oracle, 2e-3 against the emulation.
The gradient bar against FP64 is the floor that BF16 rounding itself sets:
three back-propagation stages with a relative error of 2^-9 per element,
amplified by cancellation in sums over the batch; the emulation, which has no
kernel in it, is 3.5e-2 from FP64 for the first layer at B = 64 and 1.7e-2 at
B = 1100."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

DIMS = (3, 256, 256, 256, 37)


@pytest.fixture(scope="module")
def cv():
    import paper_2507_22901_amd as cv
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    cv.lib()
    return cv


def bf(a):
    """Round to BF16 (nearest even) and back to FP32."""
    return torch.as_tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float32)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def oracle_weights(cv, flat, dims):
    """Weights as the kernels see them: BF16 for every matrix-core layer."""
    Ws, bs = cv.split_params(flat, dims)
    Ws = [Ws[0].astype(np.float64)] + [bf(w).double().numpy() for w in Ws[1:]]
    return Ws, [b.astype(np.float64) for b in bs]


def emulate(cv, flat, dims, x, gout=None, omega0=0.0):
    """FP32 forward (and backward) rounding where the kernels round."""
    Ws, bs = cv.split_params(torch.from_numpy(flat), dims)
    L = len(dims) - 1
    x = torch.as_tensor(x, dtype=torch.float32)
    z1 = x @ Ws[0].T + bs[0]
    H = [None, bf(torch.sin(omega0 * z1) if omega0 > 0 else torch.relu(z1))]
    for l in range(1, L - 1):
        H.append(bf(torch.relu(H[l] @ bf(Ws[l]).T + bs[l])))
    out = H[L - 1] @ bf(Ws[L - 1]).T + bs[L - 1]
    if gout is None:
        return out, None
    G = bf(torch.as_tensor(gout, dtype=torch.float32))
    gW, gb = [None] * L, [None] * L
    for l in range(L - 1, 0, -1):
        gW[l] = G.T @ H[l]
        gb[l] = G.sum(0)
        deriv = omega0 * torch.cos(omega0 * z1) if (l == 1 and omega0 > 0) else (H[l] > 0)
        G = bf((G @ bf(Ws[l])) * deriv)
    gW[0] = G.T @ x
    gb[0] = G.sum(0)
    return out, (gW, gb)


def _net(cv, dims=DIMS, seed=0, omega0=0.0):
    m = cv.MLP(dims)
    m.set_first_sine(omega0)
    flat = cv.init_params(dims, seed, first_sine=omega0 > 0)
    # non-zero biases so that the bias paths are exercised (a sinusoidal
    # first layer already starts with them)
    Ws, bs = cv.split_params(flat, dims)
    rng = np.random.default_rng(seed + 100)
    for l, b in enumerate(bs):
        if l > 0 or omega0 == 0:
            b[:] = rng.normal(0, 0.05, b.shape)
    m.set_params(flat)
    return m, flat


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.5, 0.5, (B, 3)).astype(np.float32)
    tr = np.where(rng.random((B, 36)) < 0.6, rng.uniform(0.02, 1.0, (B, 36)), 0.0).astype(np.float32)
    tf = (rng.random(B) < 0.7).astype(np.float32)
    return x, tr, tf


@pytest.mark.parametrize("omega0", [0.0, 30.0])
@pytest.mark.parametrize("B", [1, 300, 1100])
def test_forward_matches_references(cv, oracle, B, omega0):
    m, flat = _net(cv, omega0=omega0)
    x, _, _ = _batch(B, 1)
    out = m.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    Ws, bs = oracle_weights(cv, flat, DIMS)
    ref = oracle.mlp_forward(list(DIMS), Ws, bs, x.astype(np.float64), omega0=omega0)
    assert rel(out, ref) < 2e-2
    emu, _ = emulate(cv, flat, DIMS, x, omega0=omega0)
    assert rel(out, emu.numpy()) < 2e-3
    # kept and chunked forward agree bitwise
    out2 = m.forward(torch.from_numpy(x).cuda(), keep=True).cpu().numpy()
    assert np.array_equal(out, out2)


def test_forward_rgb8_input(cv):
    m, flat = _net(cv, seed=3)
    rgb = W.random_colours(8, 777)
    a = m.forward(torch.from_numpy(rgb).cuda())
    # the kernel's own conversion: v * fl(1/255) - 1/2 in FP32
    x = torch.from_numpy(rgb.astype(np.float32) * np.float32(1.0 / 255.0) - np.float32(0.5)).cuda()
    b = m.forward(x)
    assert torch.equal(a, b)


def test_loss_matches_oracle(cv, oracle):
    m, _ = _net(cv)
    B = 1000
    rng = np.random.default_rng(4)
    out = rng.normal(0.3, 0.4, (B, 37)).astype(np.float32)
    out[:, 36] = rng.normal(0, 3, B)
    _, tr, tf = _batch(B, 4)
    loss, gout = m.loss(torch.from_numpy(out).cuda(), torch.from_numpy(tr).cuda(),
                        torch.from_numpy(tf).cuda(), 0.1)
    val, g = oracle.mlp_loss(out.astype(np.float64), tr, tf, 0.1)
    assert abs(float(loss.item()) - val) <= 1e-5 * abs(val)
    assert np.max(np.abs(gout.cpu().numpy() - g)) <= 1e-6 * np.max(np.abs(g))


@pytest.mark.parametrize("omega0", [0.0, 30.0])
@pytest.mark.parametrize("B", [64, 300, 1100])
def test_backward_matches_references(cv, oracle, B, omega0):
    m, flat = _net(cv, seed=B, omega0=omega0)
    x, tr, tf = _batch(B, B + 1)
    xd = torch.from_numpy(x).cuda()
    out = m.forward(xd, keep=True)
    loss, gout = m.loss(out, torch.from_numpy(tr).cuda(), torch.from_numpy(tf).cuda(), 0.1)
    m.backward(xd, gout)
    grads = m.grads().cpu().numpy()
    gWs, gbs = cv.split_params(grads, DIMS)
    Ws, bs = oracle_weights(cv, flat, DIMS)
    o_gW, o_gb = oracle.mlp_backward(list(DIMS), Ws, bs, x.astype(np.float64),
                                     gout.cpu().numpy().astype(np.float64), omega0=omega0)
    _, (e_gW, e_gb) = emulate(cv, flat, DIMS, x, gout.cpu(), omega0=omega0)
    for l in range(len(DIMS) - 1):
        assert rel(gWs[l], e_gW[l].numpy()) < 2e-3, ("W emu", l)
        assert rel(gbs[l], e_gb[l].numpy()) < 2e-3, ("b emu", l)
        assert rel(gWs[l], o_gW[l]) < 5e-2, ("W", l)
        assert rel(gbs[l], o_gb[l]) < 5e-2, ("b", l)


def test_small_network_and_repeatability(cv, oracle):
    dims = (3, 32, 64, 37)
    m, flat = _net(cv, dims, seed=7)
    x, tr, tf = _batch(257, 8)
    xd = torch.from_numpy(x).cuda()
    runs = []
    for _ in range(2):
        out = m.forward(xd, keep=True)
        _, gout = m.loss(out, torch.from_numpy(tr).cuda(), torch.from_numpy(tf).cuda(), 0.1)
        m.backward(xd, gout)
        runs.append(m.grads().cpu().numpy())
    assert np.array_equal(runs[0], runs[1])   # fixed-order reductions
    Ws, bs = oracle_weights(cv, flat, dims)
    o_gW, _ = oracle.mlp_backward(list(dims), Ws, bs, x.astype(np.float64),
                                  gout.cpu().numpy().astype(np.float64))
    gWs, _ = cv.split_params(runs[0], dims)
    for l in range(len(dims) - 1):
        assert rel(gWs[l], o_gW[l]) < 5e-2


def test_adam_matches_oracle(cv, oracle):
    m, flat = _net(cv, seed=11)
    x, tr, tf = _batch(512, 12)
    xd = torch.from_numpy(x).cuda()
    p, mo, vo = flat.astype(np.float64), np.zeros(len(flat)), np.zeros(len(flat))
    for t in (1, 2, 3):
        out = m.forward(xd, keep=True)
        _, gout = m.loss(out, torch.from_numpy(tr).cuda(), torch.from_numpy(tf).cuda(), 0.1)
        m.backward(xd, gout)
        g = m.grads().cpu().numpy().astype(np.float64)
        m.adam_step(1e-3, t)
        p, mo, vo = oracle.adam_step(p, g, mo, vo, t, 1e-3)
        got = m.params().cpu().numpy()
        assert np.max(np.abs(got - p)) < 1e-6 * t, t
        p = got.astype(np.float64)  # keep the two in step


def test_save_load_roundtrip(cv, tmp_path):
    m, flat = _net(cv, seed=5, omega0=30.0)
    path = str(tmp_path / "net.cvmlp")
    m.save(path)
    m2 = cv.MLP(DIMS)
    m2.load(path)
    assert m2.omega0 == 30.0
    assert torch.equal(m.params(), m2.params())
    x = torch.from_numpy(_batch(100, 6)[0]).cuda()
    assert torch.equal(m.forward(x), m2.forward(x))
    m3 = cv.MLP((3, 32, 37))
    with pytest.raises(cv.CvError):
        m3.load(path)
    # a file in the earlier format (tag CVMLP01, no omega0 field) is a ReLU
    # network
    raw = open(path, "rb").read()
    hdr = 8 + 4 + 4 * len(DIMS) + 8
    assert raw[:8] == b"CVMLP02\0"
    old = tmp_path / "net01.cvmlp"
    old.write_bytes(b"CVMLP01\0" + raw[8:hdr] + raw[hdr + 4:])
    m2.load(str(old))
    assert m2.omega0 == 0.0
    assert torch.equal(m.params(), m2.params())
    m.set_first_sine(0.0)
    assert torch.equal(m.forward(x), m2.forward(x))
    with pytest.raises(cv.CvError):
        m.set_first_sine(-1.0)
    with pytest.raises(cv.CvError):
        m.set_first_sine(float("nan"))


def test_backward_needs_kept_forward(cv):
    m, _ = _net(cv)
    x = torch.from_numpy(_batch(64, 1)[0]).cuda()
    g = torch.zeros((64, 37), device="cuda")
    m.forward(x)  # not kept
    with pytest.raises(cv.CvError):
        m.backward(x, g)


@pytest.mark.parametrize("omega0", [0.0, 30.0])
def test_train_steps_equals_single_calls(cv, omega0):
    """The library's training loop (for the surrogate's shape, the fused
    kernels: forward with the loss, backward through the layers, the weight
    gradients, the summed gradients with Adam) does what the single calls do:
    table batch, kept forward, loss, backward, Adam with the cosine rate.
    First step: the matrix-core layers' weight gradients are equal bit for bit
    (same operands, same k order, same split sums); the biases' and the input
    layer's gradients are sums over the batch in another grouping (within
    1e-5 of the largest); the losses agree to 1e-6.  Those rounding
    differences then move the two runs apart through Adam's normalised steps
    (a gradient near zero can send a parameter's step the other way): over
    five steps the losses stay within 2e-3, the median parameter within 1% of
    the learning rate and every parameter within 2 lr per step."""
    import math
    g = torch.Generator(device="cuda").manual_seed(3)
    table = torch.randint(0, 256, (1 << 24, 40), dtype=torch.uint8, device="cuda", generator=g)
    ids = torch.randint(0, 1 << 24, (5000,), dtype=torch.int32, device="cuda", generator=g)
    a, flat = _net(cv, dims=cv.SURROGATE_DIMS, seed=21, omega0=omega0)
    b = cv.MLP(cv.SURROGATE_DIMS)
    b.set_first_sine(omega0)
    b.set_params(flat)
    batch, total, dr, delta, lr0, lr1 = 1024, 5, 0.25, 0.05, 2e-3, 2e-5
    manual = []
    grads_first = None
    for k in range(total):
        x, tr, tf = b.table_batch(ids[k * batch:(k + 1) * batch], table, dr)
        out = b.forward(x, keep=True)
        loss, gout = b.loss(out, tr, tf, delta)
        b.backward(x, gout)
        if k == 0:
            grads_first = b.grads().clone()
        # the loop's schedule: double arithmetic on the FP32 rates it was given
        frac = k / (total - 1)
        f0, f1 = float(np.float32(lr0)), float(np.float32(lr1))
        lr = f1 + 0.5 * (f0 - f1) * (1.0 + math.cos(math.pi * frac))
        b.adam_step(float(np.float32(lr)), k + 1)
        manual.append(loss)
    manual = torch.cat(manual)
    losses = [a.train_steps(ids[:batch], table, dr, batch, delta, lr0, lr1, 0, total)]
    ga = a.grads()
    gws_a, gbs_a = cv.split_params(ga.cpu().numpy(), cv.SURROGATE_DIMS)
    gws_b, gbs_b = cv.split_params(grads_first.cpu().numpy(), cv.SURROGATE_DIMS)
    for l in range(1, 4):
        assert np.array_equal(gws_a[l], gws_b[l]), l
    scale = max(np.abs(grads_first.cpu().numpy()).max(), 1e-30)
    for l in range(4):
        assert np.max(np.abs(gbs_a[l] - gbs_b[l])) <= 1e-5 * scale, l
    assert np.max(np.abs(gws_a[0] - gws_b[0])) <= 1e-5 * scale
    assert abs(float(losses[0][0]) - float(manual[0])) <= 1e-6 * abs(float(manual[0]))
    losses.append(a.train_steps(ids[batch:], table, dr, batch, delta, lr0, lr1, 1, total))
    losses = torch.cat(losses)
    assert torch.allclose(losses, manual, rtol=2e-3, atol=0.0)
    pa, pb = a.params(), b.params()
    d = torch.abs(pa - pb)
    assert float(d.max()) <= 2 * lr0 * total
    assert float(d.median()) <= 1e-2 * lr0


@pytest.mark.parametrize("omega0", [0.0, 30.0])
@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 70001])
def test_fused_inference_equals_layer_by_layer(cv, n, omega0):
    """8-bit colours through the surrogate's shape take the fused kernel
    (activations in LDS); a kept forward and FP32 inputs take the
    layer-by-layer kernels.  All round at the same points (the input
    conversion v * fl(1/255) - 1/2 with two roundings, as numpy does it), so
    the outputs are equal bit for bit."""
    m, _ = _net(cv, dims=cv.SURROGATE_DIMS, seed=5, omega0=omega0)
    rgb = W.random_colours(9, n)
    a = m.forward(torch.from_numpy(rgb).cuda())
    k = m.forward(torch.from_numpy(rgb).cuda(), keep=True)
    x = torch.from_numpy(rgb.astype(np.float32) * np.float32(1.0 / 255.0) - np.float32(0.5)).cuda()
    b = m.forward(x)
    assert torch.equal(a, k) and torch.equal(k, b)


def _mix64(z):
    M = (1 << 64) - 1
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def _feistel_order(n, key):
    """The training order from its definition: four Feistel rounds on 2h-bit
    values, round r xor-ing mix64(R + k_r) mod 2^h into L, cycle-walked back
    into [0, n)."""
    M = (1 << 64) - 1
    h = 1
    while (1 << (2 * h)) < n:
        h += 1
    ks = [_mix64((key + (r + 1) * 0x9E3779B97F4A7C15) & M) for r in range(4)]
    mask = (1 << h) - 1

    def pi(v):
        L, R = v >> h, v & mask
        for k in ks:
            L, R = R, L ^ (_mix64((R + k) & M) & mask)
        return (L << h) | R

    out = []
    for i in range(n):
        v = pi(i)
        while v >= n:
            v = pi(v)
        out.append(v)
    return out


@pytest.mark.parametrize("n,key", [(1, 0), (2, 5), (7, 1), (1000, 3), (4097, (1 << 32) + 2)])
def test_permute_ids_matches_definition(cv, n, key):
    ids = torch.arange(10, 10 + n, dtype=torch.int32, device="cuda")
    got = cv.permute_ids(ids, key).cpu().numpy()
    want = 10 + np.array(_feistel_order(n, key))
    assert np.array_equal(got, want)


def test_permute_ids_is_a_shuffle(cv):
    n = 15_101_294   # the training colours of the whole-cube 90/10 split
    ids = torch.arange(n, dtype=torch.int32, device="cuda") * 3
    a = cv.permute_ids(ids, 1)
    b = cv.permute_ids(ids, 2)
    assert torch.equal(torch.sort(a).values, ids)       # a permutation
    assert torch.equal(cv.permute_ids(ids, 1), a)       # the same key, the same order
    fixed = int((a == ids).sum())
    assert fixed < 100                                  # about one expected
    assert int((a == b).sum()) < 100
    # neighbours in the output come from far apart in the input
    d = torch.abs(a[1:].double() - a[:-1].double()) / 3
    assert float(d.median()) > n / 8
    with pytest.raises(cv.CvError):   # in place is refused
        cv._check(cv.lib().cv_permute_ids(cv.context().handle, cv._dptr(ids), n, 1, cv._dptr(ids), None))


# --------------------------------------------------------------------------
# Layer by layer, element by element: the FP64 oracle is given each layer's
# own input as the kernels hold it (x for the first layer, the kept BF16
# activations after it), so the comparison sees only the kernels' FP32
# accumulation and their single BF16 rounding of each activation.  An element
# of a product sum_i a_i b_i is held to tol * sum_i |a_i b_i|.

def _elementwise(got, ref, scale, tol, what):
    err = np.abs(np.asarray(got, np.float64) - ref)
    lim = tol * np.asarray(scale, np.float64) + 1e-30
    bad = err > lim
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {bad.size} elements off; worst "
                           f"{float(np.max(err / lim)):.3g} x the bound")


def _layer_io(cv, m, flat, x, omega0):
    L = len(DIMS) - 1
    B = x.shape[0]
    H = [x.astype(np.float64)] + [m.hidden(l, B).cpu().numpy().astype(np.float64) for l in range(1, L)]
    Ws, bs = oracle_weights(cv, flat, DIMS)
    return L, H, Ws, bs


@pytest.mark.parametrize("omega0", [0.0, 30.0])
def test_layers_elementwise_against_oracle(cv, oracle, omega0):
    m, flat = _net(cv, seed=31, omega0=omega0)
    B = 700
    x, tr, tf = _batch(B, 32)
    xd = torch.from_numpy(x).cuda()
    outd = m.forward(xd, keep=True)
    out = outd.cpu().numpy().astype(np.float64)
    L, H, Ws, bs = _layer_io(cv, m, flat, x, omega0)
    z1 = None
    for l in range(L):
        z = oracle.mlp_forward([DIMS[l], DIMS[l + 1]], [Ws[l]], [bs[l]], H[l])
        scale = np.abs(H[l]) @ np.abs(Ws[l]).T + np.abs(bs[l])
        if l == 0:
            z1 = z
        if l == L - 1:
            _elementwise(out, z, scale, 1e-5, "output layer")
            continue
        sine = l == 0 and omega0 > 0
        a = np.sin(omega0 * z) if sine else np.maximum(z, 0.0)
        # the FP32 pre-activation (error <= 1e-5 x scale, times omega0 through
        # the sine) and one BF16 rounding (<= 2^-8 |a|)
        _elementwise(H[l + 1], a, 2.0 ** -8 / 1e-5 * np.abs(a) + (omega0 if sine else 1.0) * scale, 1e-5,
                     f"hidden layer {l + 1}")
    # backward: the output gradient as the kernels read it (BF16), then the
    # chain through the kernels' own activations
    _, gout = m.loss(outd, torch.from_numpy(tr).cuda(), torch.from_numpy(tf).cuda(), 0.1)
    m.backward(xd, gout)
    gWs, gbs = cv.split_params(m.grads().cpu().numpy(), DIMS)
    G = bf(gout.cpu()).double().numpy()
    for l in range(L - 1, -1, -1):
        (gW_ref,), (gb_ref,) = oracle.mlp_backward([DIMS[l], DIMS[l + 1]], [Ws[l]], [bs[l]], H[l], G)
        sW = np.abs(G).T @ np.abs(H[l])
        sb = np.abs(G).sum(0)
        # the last layer reads exactly the kernels' operands (FP32 sums only);
        # below it the host's chain may round a few BF16 gradients the other
        # way, each moving a term by at most 2^-8 of itself
        tol = 1e-5 if l == L - 1 else 1e-2
        _elementwise(gWs[l], gW_ref, sW, tol, f"weight gradient {l}")
        _elementwise(gbs[l], gb_ref, sb, tol, f"bias gradient {l}")
        if l == 0:
            break
        gin = oracle.linear_input_grad(Ws[l], G)
        if l == 1 and omega0 > 0:
            deriv = omega0 * np.cos(omega0 * z1)
        else:
            deriv = (H[l] > 0).astype(np.float64)
        G = bf(torch.from_numpy(gin * deriv)).double().numpy()


def test_exact_bf16_network_equals_oracle(cv, oracle):
    """Weights, biases, inputs and output gradients chosen so that every
    activation and every back-propagated gradient is a small integer, which
    BF16 holds exactly and FP32 sums exactly: the kernels must then give the
    FP64 oracle's outputs and gradients to 1e-5 (in fact exactly).  This checks
    the kernels' arithmetic without the BF16 noise floor (index, layout and
    transposition mistakes show at once)."""
    rng = np.random.default_rng(41)
    dims = DIMS
    Ws, bs = [], []
    for l in range(len(dims) - 1):
        din, dout = dims[l], dims[l + 1]
        W = np.zeros((dout, din))
        k = 3 if l == 0 else 4   # non-zeros per row
        for o in range(dout):
            cols_ = rng.choice(din, min(k, din), replace=False)
            W[o, cols_] = rng.choice([-1.0, 1.0], len(cols_))
        Ws.append(W)
        bs.append(rng.integers(-2, 3, dout).astype(np.float64))
    flat = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in zip(Ws, bs)]).astype(np.float32)
    m = cv.MLP(dims)
    m.set_first_sine(0.0)
    m.set_params(flat)
    B = 96
    x = rng.integers(-2, 3, (B, 3)).astype(np.float32)
    xd = torch.from_numpy(x).cuda()
    out = m.forward(xd, keep=True).cpu().numpy().astype(np.float64)
    ref = oracle.mlp_forward(list(dims), Ws, bs, x.astype(np.float64))
    # every hidden activation is a small integer (exact in BF16: below 256)
    for l in range(1, len(dims) - 1):
        h = m.hidden(l, B).cpu().numpy()
        assert np.array_equal(h, np.rint(h)) and np.abs(h).max() < 256, l
    assert np.max(np.abs(out - ref)) <= 1e-5 * np.abs(ref).max()
    gout = rng.integers(-1, 2, (B, dims[-1])).astype(np.float32)
    m.backward(xd, torch.from_numpy(gout).cuda())
    gWs, gbs = cv.split_params(m.grads().cpu().numpy(), dims)
    o_gW, o_gb = oracle.mlp_backward(list(dims), Ws, bs, x.astype(np.float64), gout.astype(np.float64))
    for l in range(len(dims) - 1):
        assert np.max(np.abs(gWs[l] - o_gW[l])) <= 1e-5 * max(np.abs(o_gW[l]).max(), 1.0), l
        assert np.max(np.abs(gbs[l] - o_gb[l])) <= 1e-5 * max(np.abs(o_gb[l]).max(), 1.0), l
    assert max(np.abs(g).max() for g in o_gW) > 10  # the check is not vacuous
