"""GPU network (BF16 weights on the MFMA, FP32 accumulate, activations carried
as hi + lo BF16 pairs) against the FP64 oracle on the same BF16-rounded
weights.  Bars: per-tensor relative error (2-norm) <= 1e-2 and cosine
similarity >= 0.999 for the forward logits and every gradient tensor."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_1210_5128_amd import datagen

pytestmark = pytest.mark.gpu

N_PARAM = 17793
H = 128


@pytest.fixture(scope="module")
def bnos():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1210_5128_amd import bnos as b
    return b


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def oracle_params(p32):
    """The weights the device computes with: W1, W2, w3 in BF16, biases FP32."""
    p = p32.astype(np.float64).copy()
    for a, b in [(0, H * 8), (H * 8 + H, H * 8 + H + H * H), (H * 8 + H + H * H + H, H * 8 + H + H * H + 2 * H)]:
        p[a:b] = bf16_round(p32[a:b])
    return p


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def sample_inputs(R, n, seed):
    rng = np.random.default_rng(seed)
    feats = rng.standard_normal((R, n, 8)).astype(np.float32) * np.array([0.3, 40, 5, 2, 2, 30, 30, 4], np.float32)
    feats += np.array([0.5, -900, 3, 0, 0, -600, -800, 20], np.float32)
    pairs = np.stack([rng.choice(n, 2, replace=False) for _ in range(R)]).astype(np.int32)
    return feats, pairs


def test_forward_matches_oracle(bnos):
    R, n = 24, 37
    feats, _ = sample_inputs(R, n, 1)
    p32 = datagen.mlp_params(5).astype(np.float32)
    mu = feats.reshape(-1, 8).mean(axis=0)
    sd = feats.reshape(-1, 8).std(axis=0)
    m = bnos.Mlp()
    m.set_params(p32, mu, sd)
    f = torch.from_numpy(feats).cuda()
    out = torch.empty((R, n), dtype=torch.float32, device="cuda")
    m.forward(f, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    po = oracle_params(p32)
    want = np.stack([oracle.mlp_forward(po, (feats[s].astype(np.float64) - mu) / sd) for s in range(R)])
    print(f"forward logits: rel {rel(got, want):.3e}, cos {cos(got.ravel(), want.ravel()):.9f}", flush=True)
    assert rel(got, want) < 1e-2, rel(got, want)
    assert cos(got.ravel(), want.ravel()) > 0.9999
    # determinism
    out2 = torch.empty_like(out)
    m.forward(f, out2)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    m.free()


def hilo(x):
    """The two BF16 halves the kernels feed the matrix cores for an FP32 activation x."""
    x32 = np.asarray(x, dtype=np.float32)
    h = bf16_round(x32)
    lo = bf16_round((x32.astype(np.float64) - h).astype(np.float32))
    return h, lo


def emulate_grad(p32, mu, sd, feats, pairs, eps):
    """FP64 replay of the kernel's arithmetic: BF16 weights, every activation
    operand split into BF16 hi + lo, products of two activations as
    hi*hi + hi*lo + lo*hi (+ lo*lo for the first layer's weight gradient)."""
    po = oracle_params(p32)
    W1 = po[:H * 8].reshape(H, 8)
    b1 = po[H * 8:H * 8 + H]
    W2 = po[H * 8 + H:H * 8 + H + H * H].reshape(H, H)
    b2 = po[H * 8 + H + H * H:H * 8 + 2 * H + H * H]
    w3 = po[H * 8 + 2 * H + H * H:N_PARAM - 1]
    b3 = po[-1]
    rsd = (np.float32(1.0) / sd.astype(np.float32))
    g = np.zeros(N_PARAM)
    gW1 = np.zeros((H, 8)); gb1 = np.zeros(H); gW2 = np.zeros((H, H)); gb2 = np.zeros(H); gw3 = np.zeros(H)
    gb3 = 0.0
    loss = 0.0
    R, n = feats.shape[0], feats.shape[1]
    for s in range(R):
        zh, zl = hilo((feats[s] - mu.astype(np.float32)) * rsd)
        h1 = np.maximum((zh + zl) @ W1.T + b1, 0).astype(np.float32)
        h1h, h1l = hilo(h1)
        h2 = np.maximum((h1h + h1l) @ W2.T + b2, 0)
        lg = (h2 @ w3 + b3).astype(np.float32).astype(np.float64)
        p = np.exp(lg - lg.max()); p /= p.sum()
        a, b = int(pairs[s, 0]), int(pairs[s, 1])
        pa, pb = p[a], p[b]
        Q = pa * pb * (1 / (1 - pa) + 1 / (1 - pb))
        q = (1 - eps) * Q + eps * 2 / (n * (n - 1))
        ga = pa * pb * (1 / (1 - pa) ** 2 + 1 / (1 - pb))
        gb = pb * pa * (1 / (1 - pb) ** 2 + 1 / (1 - pa))
        dQ = -p * (ga + gb)
        dQ[a] += ga
        dQ[b] += gb
        dl = (-(1 - eps) * dQ / q).astype(np.float32).astype(np.float64)
        loss += -np.log(q)
        d2f = np.where(h2 > 0, dl[:, None] * w3[None, :], 0.0)
        d2h, d2l = hilo(d2f)
        gw3 += dl @ h2
        gb2 += d2f.sum(axis=0)
        gb3 += dl.sum()
        gW2 += d2h.T @ h1h + d2h.T @ h1l + d2l.T @ h1h
        dpre1 = np.where(h1h != 0, (d2h + d2l) @ W2, 0.0)
        gb1 += dpre1.sum(axis=0)
        dph, dpl = hilo(dpre1)
        gW1 += (dph + dpl).T @ (zh + zl)
    g[:H * 8] = gW1.ravel(); g[H * 8:H * 8 + H] = gb1
    g[H * 8 + H:H * 8 + H + H * H] = gW2.ravel(); g[H * 8 + H + H * H:H * 8 + 2 * H + H * H] = gb2
    g[H * 8 + 2 * H + H * H:N_PARAM - 1] = gw3; g[-1] = gb3
    return g / R, loss / R


@pytest.mark.parametrize("n", [5, 20, 60, 64])
def test_gradient_matches_oracle(bnos, n):
    R = 40
    feats, pairs = sample_inputs(R, n, 2 + n)
    p32 = datagen.mlp_params(9).astype(np.float32)
    mu = feats.reshape(-1, 8).mean(axis=0)
    sd = feats.reshape(-1, 8).std(axis=0)
    m = bnos.Mlp()
    m.set_params(p32, mu, sd)
    g = torch.empty(N_PARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    m.grad(torch.from_numpy(feats).cuda(), torch.from_numpy(pairs).cuda(), g, loss, eps=0.1)
    got = g.cpu().numpy().astype(np.float64)
    po = oracle_params(p32)
    want = np.zeros(N_PARAM)
    wl = 0.0
    for s in range(R):
        z = (feats[s].astype(np.float64) - mu) / sd
        l, gs = oracle.mlp_loss_grad(po, z, int(pairs[s, 0]), int(pairs[s, 1]), 0.1)
        want += gs / R
        wl += l / R
    sl = {"W1": slice(0, H * 8), "b1": slice(H * 8, H * 8 + H), "W2": slice(H * 8 + H, H * 8 + H + H * H),
          "b2": slice(H * 8 + H + H * H, H * 8 + 2 * H + H * H), "w3": slice(H * 8 + 2 * H + H * H, N_PARAM - 1)}
    errs = {k: (rel(got[s_], want[s_]), cos(got[s_], want[s_])) for k, s_ in sl.items()}
    emu, _ = emulate_grad(p32, mu, sd, feats, pairs, 0.1)
    eerr = {k: rel(got[s_], emu[s_]) for k, s_ in sl.items()}
    print(f"n={n}: loss {loss.item():.9f} vs {wl:.9f}; rel / cos per tensor vs the FP64 oracle: {errs}; "
          f"rel vs the emulated kernel: {eerr}", flush=True)
    assert abs(loss.item() - wl) <= 1e-4 * abs(wl), (loss.item(), wl)
    # (1) the FP64 oracle on the same BF16 weights: the contract bar, every tensor
    for name, s_ in sl.items():
        assert errs[name][0] <= 1e-2, (name, errs[name])
        assert errs[name][1] >= 0.999, (name, errs[name])
    assert abs(got[-1] - want[-1]) <= 1e-2 * max(abs(want[-1]), 1e-3)
    # (2) the kernel's own arithmetic (hi/lo operands), up to FP32 accumulation order
    for name, s_ in sl.items():
        assert eerr[name] < 1e-3, (name, "emulated", eerr[name])
    assert abs(got[-1] - emu[-1]) <= 1e-3 * max(abs(emu[-1]), 1e-3)
    m.free()


def test_fit_norm_and_params_roundtrip(bnos):
    feats, _ = sample_inputs(50, 30, 3)
    m = bnos.Mlp()
    m.fit_norm(torch.from_numpy(feats).cuda())
    p, mu, sd = m.get_params()
    flat = feats.reshape(-1, 8).astype(np.float64)
    np.testing.assert_allclose(mu, flat.mean(axis=0), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(sd, flat.std(axis=0), rtol=1e-5)
    p32 = datagen.mlp_params(4).astype(np.float32)
    m.set_params(p32)
    p2, _, _ = m.get_params()
    assert np.array_equal(p2, p32)
    m.free()


def test_training_fits_a_teacher(bnos):
    # samples whose pairs are drawn from a teacher network's q; the student's
    # loss must fall toward the teacher's cross-entropy
    n, R = 12, 4096
    rng = np.random.default_rng(8)
    feats = rng.standard_normal((R, n, 8)).astype(np.float32)
    teacher = datagen.mlp_params(21, scale=2.0)
    pairs = np.zeros((R, 2), dtype=np.int32)
    ent = 0.0
    for s in range(R):
        lg = oracle.mlp_forward(teacher, feats[s].astype(np.float64))
        qs = []
        idx = []
        for a in range(n):
            for b in range(a + 1, n):
                qs.append(np.exp(oracle.pair_logq(lg, a, b, 0.1)))
                idx.append((a, b))
        qs = np.array(qs) / np.sum(qs)
        k = rng.choice(len(qs), p=qs)
        pairs[s] = idx[k]
        ent += -np.log(qs[k]) / R
    m = bnos.Mlp()
    m.set_params(datagen.mlp_params(22, scale=0.5).astype(np.float32), np.zeros(8, np.float32), np.ones(8, np.float32))
    f = torch.from_numpy(feats).cuda()
    pr = torch.from_numpy(pairs).cuda()
    g = torch.empty(N_PARAM, dtype=torch.float32, device="cuda")
    l0 = torch.empty(1, dtype=torch.float64, device="cuda")
    m.grad(f, pr, g, l0)
    trace = torch.zeros(8 * 16, dtype=torch.float32, device="cuda")
    m.train(f, pr, epochs=8, batch=256, lr=3e-3, seed=1, loss_trace=trace)
    l1 = torch.empty(1, dtype=torch.float64, device="cuda")
    m.grad(f, pr, g, l1)
    uniform = np.log(n * (n - 1) / 2)
    assert l1.item() < l0.item() - 0.3, (l0.item(), l1.item())
    assert l1.item() < uniform - 0.2
    assert l1.item() > ent - 0.1          # cannot beat the teacher by much on its own samples
    tr = trace.cpu().numpy()
    assert np.all(np.isfinite(tr)) and tr[-16:].mean() < tr[:16].mean()
    m.free()
