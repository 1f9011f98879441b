"""The packed layout of the MLP surrogate, checked on the CPU.

The packer (C ABI, syn_mlp_pack) stores each layer as the A-operand fragments
of v_mfma_f32_32x32x16_f16 with the input features permuted into the order in
which the previous layer's accumulator rows sit in the lanes.  This test
undoes the packing with the hardware operand layout (lane l, element i of a
k-step t holds row l % 32 and column 16 t + 8 (l // 32) + i; accumulator
register r of lane l holds row (r % 4) + 8 (r // 4) + 4 (l // 32)), runs the
network that way in numpy, and compares with the plain PyTorch model.
"""
import numpy as np
import pytest
import torch

from paper_2410_01136_amd import inputs as I


@pytest.fixture(scope="module")
def S():
    from paper_2410_01136_amd import surrogate
    return surrogate


def f16_bits_to_f32(u16):
    return u16.view(np.float16).astype(np.float32)


OFF_FOURIER, OFF_W0 = 0, 256
W0_BYTES = 4 * 2 * 64 * 8 * 2
HID_BYTES = 4 * 8 * 64 * 8 * 2
OFF_W1 = OFF_W0 + W0_BYTES
OFF_WOUT = OFF_W1 + 3 * HID_BYTES
OFF_BIAS = OFF_WOUT + 8 * 64 * 8 * 2
OFF_BOUT = OFF_BIAS + 4 * 128 * 4


def acc_row(r, h):
    return (r % 4) + 8 * (r // 4) + 4 * h


def unpack_layer(P, off, n_rb, n_t):
    """A matrix [32 n_rb][16 n_t] as seen by the matrix unit (column order = k)."""
    frag = f16_bits_to_f32(np.frombuffer(P, dtype=np.uint16, count=n_rb * n_t * 64 * 8,
                                          offset=off)).reshape(n_rb, n_t, 64, 8)
    A = np.zeros((32 * n_rb, 16 * n_t), dtype=np.float64)
    for rb in range(n_rb):
        for t in range(n_t):
            for l in range(64):
                for i in range(8):
                    A[32 * rb + l % 32, 16 * t + 8 * (l // 32) + i] = frag[rb, t, l, i]
    return A


def feature_of_k(k):
    t, rem = divmod(k, 16)
    h, i = divmod(rem, 8)
    return 32 * (t // 2) + 16 * (t % 2) + 8 * (i // 4) + 4 * h + (i % 4)


def test_packed_network_matches_model(S):
    import math
    torch.manual_seed(0)
    model = S.FieldMLP(I.BOX_LO, I.BOX_HI, seed=11)
    # non-trivial output de-standardisation
    model.out_scale.copy_(torch.tensor([3.0, 3.0, 3.0, 0.7, 0.2]))
    model.out_shift.copy_(torch.tensor([0.0, 0.0, 0.0, -4.0, -10.0]))
    P = S.pack(model, device="cpu").numpy().tobytes()
    fq = np.frombuffer(P, dtype=np.float32, count=48, offset=OFF_FOURIER).reshape(16, 3)
    np.testing.assert_array_equal(fq, model.fourier.numpy())
    A0 = unpack_layer(P, OFF_W0, 4, 2)
    Ah = [unpack_layer(P, OFF_W1 + j * HID_BYTES, 4, 8) for j in range(3)]
    Ao = unpack_layer(P, OFF_WOUT, 1, 8)
    bias = np.frombuffer(P, dtype=np.float32, count=4 * 128, offset=OFF_BIAS).reshape(4, 4, 2, 16)
    bout = np.frombuffer(P, dtype=np.float32, count=5, offset=OFF_BOUT)
    # biases in accumulator order
    e = model.export()
    # the packer rounds to FP16 as numpy does (round to nearest even)
    np.testing.assert_array_equal(A0, e["w_in"].astype(np.float16).astype(np.float64))
    for layer in range(4):
        b = e["b_in"] if layer == 0 else e["b_h"][layer - 1]
        for rb in range(4):
            for h in range(2):
                for r in range(16):
                    assert bias[layer, rb, h, r] == np.float32(b[32 * rb + acc_row(r, h)])
    # run 200 points through the unpacked matrices (feature order = k order)
    rng = np.random.default_rng(3)
    r = rng.uniform(I.BOX_LO, I.BOX_HI, size=(200, 3))
    # features exactly as the reference computes them (FP32), so both start from
    # identical FP16 inputs; later layers differ only by summation order
    rt = torch.from_numpy(r).float()
    xt = 2.0 * (rt - model.lo) / (model.hi - model.lo) - 1.0
    tt = xt @ torch.from_numpy(fq).T
    feats = torch.cat([torch.sin(2 * math.pi * tt), torch.cos(2 * math.pi * tt)], 1).numpy()
    f16 = lambda a: a.astype(np.float16).astype(np.float64)
    # the kernel's bias and gate (FP32 bias in the sum, rounded to FP16, FP16 gate)
    act = lambda acc, b: S.layer_f16(torch.from_numpy(acc.astype(np.float32)),
                                     torch.from_numpy(b.astype(np.float32))).numpy().astype(np.float64)
    h = act(f16(feats) @ A0.T, e["b_in"])  # layer 0 columns are in natural feature order
    perm = np.array([feature_of_k(k) for k in range(128)])
    for j in range(3):
        h = act(h[:, perm] @ Ah[j].T, e["b_h"][j])
    o = h[:, perm] @ Ao.T  # 32 rows: outputs at {0,1,2,3,8} and {4,5,6,7,12}
    for rows in ([0, 1, 2, 3, 8], [4, 5, 6, 7, 12]):
        out = o[:, rows] + bout
        ref = S.reference_eval(model, torch.from_numpy(r).float()).numpy()
        ref_raw = np.concatenate([ref[:, :3], np.log(ref[:, 3:5])], 1)
        # FP16 rounding-boundary flips stay at the 1e-3 level; a misplaced weight or
        # permutation would give errors of the order of the outputs themselves
        err = np.abs(out - ref_raw)
        assert np.all(err <= 5e-3 * np.abs(ref_raw).max(0)), err.max(0)
        assert np.median(err / np.abs(ref_raw).max(0)) < 1e-4
    # the unused output rows are empty
    others = [k for k in range(32) if k not in (0, 1, 2, 3, 8, 4, 5, 6, 7, 12)]
    assert np.all(Ao[others] == 0)


def test_f16_reference_close_to_fp32_model(S):
    model = S.FieldMLP(I.BOX_LO, I.BOX_HI, seed=12)
    r = torch.from_numpy(np.random.default_rng(4).uniform(I.BOX_LO, I.BOX_HI, (500, 3))).float()
    ref = S.reference_eval(model, r)
    full = model(r)
    raw = torch.cat([ref[:, :3], torch.log(ref[:, 3:5])], 1)
    assert torch.allclose(raw, full, rtol=0.05, atol=0.05 * full.abs().max().item())
