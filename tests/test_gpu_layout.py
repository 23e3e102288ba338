"""In-bounds checks of the MFMA builtins' lane layouts and of the FP8/BF16
conversions the fused kernel relies on (one wave per probe)."""
import ctypes
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

SO = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2510_24380_amd", "probe",
                  "libmfma_probe.so")


def e4m3_table():
    """Values of the 256 OCP E4M3 (FN) codes; NaN for 0x7f and 0xff."""
    vals = np.zeros(256, np.float64)
    for b in range(256):
        s, e, m = b >> 7, (b >> 3) & 15, b & 7
        if e == 15 and m == 7:
            vals[b] = np.nan
        elif e == 0:
            vals[b] = (-1) ** s * 2.0 ** -6 * (m / 8)
        else:
            vals[b] = (-1) ** s * 2.0 ** (e - 7) * (1 + m / 8)
    return vals


@pytest.fixture(scope="module")
def probe():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = ctypes.CDLL(SO)
    lib.probe_mfma.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.probe_cvt.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]
    lib.probe_mfma_fp8_scaled.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    return lib


def run(probe, kind, a_regs, b_regs):
    a = torch.from_numpy(np.ascontiguousarray(a_regs)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(b_regs)).cuda()
    d = torch.zeros(256, dtype=torch.float32, device="cuda")
    assert probe.probe_mfma(kind, a.data_ptr(), b.data_ptr(), d.data_ptr()) == 0
    regs = d.cpu().numpy().reshape(64, 4)
    D = np.zeros((16, 16))
    for l in range(64):
        for v in range(4):
            D[4 * (l // 16) + v, l % 16] = regs[l, v]
    return D


def run32(probe, kind, a_regs, b_regs):
    """32x32 shapes: lane l holds accumulator v at row 8 (v // 4) + 4 (l // 32) + v % 4,
    column l % 32."""
    a = torch.from_numpy(np.ascontiguousarray(a_regs)).cuda()
    b = torch.from_numpy(np.ascontiguousarray(b_regs)).cuda()
    d = torch.zeros(64 * 16, dtype=torch.float32, device="cuda")
    assert probe.probe_mfma(kind, a.data_ptr(), b.data_ptr(), d.data_ptr()) == 0
    regs = d.cpu().numpy().reshape(64, 16)
    D = np.zeros((32, 32))
    for l in range(64):
        for v in range(16):
            D[8 * (v // 4) + 4 * (l // 32) + v % 4, l % 32] = regs[l, v]
    return D, regs


def test_mfma_f32_16x16x4(probe):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((16, 4)).astype(np.float32)
    B = rng.standard_normal((4, 16)).astype(np.float32)
    a = np.array([A[l % 16, l // 16] for l in range(64)], np.float32)
    b = np.array([B[l // 16, l % 16] for l in range(64)], np.float32)
    D = run(probe, 0, a, b)
    np.testing.assert_allclose(D, A.astype(np.float64) @ B, rtol=1e-5, atol=1e-5)


def test_mfma_bf16_16x16x32(probe):
    rng = np.random.default_rng(2)
    def bf16_round(x):  # values exactly representable in bf16
        u = x.astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
        return u.view(np.float32)
    A = bf16_round(rng.standard_normal((16, 32)))
    B = bf16_round(rng.standard_normal((32, 16)))
    a = np.zeros((64, 8), np.uint16)
    b = np.zeros((64, 8), np.uint16)
    for l in range(64):
        for e in range(8):
            k = 8 * (l // 16) + e
            a[l, e] = A[l % 16, k].view(np.uint32) >> 16
            b[l, e] = B[k, l % 16].view(np.uint32) >> 16
    D = run(probe, 1, a, b)
    np.testing.assert_allclose(D, A.astype(np.float64) @ B, rtol=1e-5, atol=1e-4)


def test_mfma_bf16_32x32x16(probe):
    """A: lane l holds row l % 32, k = 8 (l // 32) + e; B: column l % 32, same k."""
    rng = np.random.default_rng(5)
    def bf16_round(x):
        u = x.astype(np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
        return u.view(np.float32)
    A = bf16_round(rng.standard_normal((32, 16)))
    B = bf16_round(rng.standard_normal((16, 32)))
    a = np.zeros((64, 8), np.uint16)
    b = np.zeros((64, 8), np.uint16)
    for l in range(64):
        for e in range(8):
            k = 8 * (l // 32) + e
            a[l, e] = A[l % 32, k].view(np.uint32) >> 16
            b[l, e] = B[k, l % 32].view(np.uint32) >> 16
    D, regs = run32(probe, 3, a, b)
    if not np.allclose(D, A.astype(np.float64) @ B, rtol=1e-5, atol=1e-4):
        print("lane 0 regs", regs[0], "lane 32 regs", regs[32])
    np.testing.assert_allclose(D, A.astype(np.float64) @ B, rtol=1e-5, atol=1e-4)


def test_mfma_fp8_32x32x64(probe):
    """A: lane l holds row l % 32, k = 32 (l // 32) + e; B: column l % 32, same k."""
    rng = np.random.default_rng(6)
    tab = e4m3_table()
    okn = np.where(np.isfinite(tab) & (np.abs(tab) <= 8) & (np.abs(tab) >= 2.0 ** -6))[0]
    ca = rng.choice(okn, (32, 64)).astype(np.uint8)
    cb = rng.choice(okn, (64, 32)).astype(np.uint8)
    A, B = tab[ca], tab[cb]
    a = np.zeros((64, 32), np.uint8)
    b = np.zeros((64, 32), np.uint8)
    for l in range(64):
        for e in range(32):
            k = 32 * (l // 32) + e
            a[l, e] = ca[l % 32, k]
            b[l, e] = cb[k, l % 32]
    D, regs = run32(probe, 4, a, b)
    e_norm = float(np.max(np.abs(D - A @ B) / (np.abs(A) @ np.abs(B))))
    print(f"fp8 32x32x64 mfma, normal inputs: max error / sum|ab| {e_norm:.2e}")
    assert e_norm < 2e-3


def test_mfma_fp8_32x32x64_block_scales(probe):
    """The scaled form multiplies the product by 2^(sa - 127) 2^(sb - 127) (E8M0
    scales), exactly: the FP8 kernel applies the GEMM's power-of-two scale this
    way instead of one multiply per activation."""
    rng = np.random.default_rng(7)
    tab = e4m3_table()
    okn = np.where(np.isfinite(tab) & (np.abs(tab) <= 8) & (np.abs(tab) >= 2.0 ** -6))[0]
    ca = rng.choice(okn, (32, 64)).astype(np.uint8)
    cb = rng.choice(okn, (64, 32)).astype(np.uint8)
    a = np.zeros((64, 32), np.uint8)
    b = np.zeros((64, 32), np.uint8)
    for l in range(64):
        for e in range(32):
            k = 32 * (l // 32) + e
            a[l, e] = ca[l % 32, k]
            b[l, e] = cb[k, l % 32]
    D, regs = run32(probe, 4, a, b)
    for sa, sb in [(127, 127), (130, 127), (127 - 9, 127), (131, 127 - 6)]:
        at = torch.from_numpy(np.ascontiguousarray(a)).cuda()
        bt = torch.from_numpy(np.ascontiguousarray(b)).cuda()
        d = torch.zeros(64 * 16, dtype=torch.float32, device="cuda")
        assert probe.probe_mfma_fp8_scaled(at.data_ptr(), bt.data_ptr(), d.data_ptr(), sa, sb) == 0
        got = d.cpu().numpy().reshape(64, 16)
        want = (regs.astype(np.float64) * 2.0 ** (sa - 127 + sb - 127)).astype(np.float32)
        assert np.array_equal(got, want), f"scales {sa}, {sb}"


def test_mfma_fp8_16x16x128(probe):
    rng = np.random.default_rng(3)
    tab = e4m3_table()
    ok = np.where(np.isfinite(tab) & (np.abs(tab) <= 8))[0]
    ca = rng.choice(ok, (16, 128)).astype(np.uint8)
    cb = rng.choice(ok, (128, 16)).astype(np.uint8)
    A, B = tab[ca], tab[cb]
    a = np.zeros((64, 32), np.uint8)
    b = np.zeros((64, 32), np.uint8)
    for l in range(64):
        for e in range(32):
            k = 32 * (l // 16) + e
            a[l, e] = ca[l % 16, k]
            b[l, e] = cb[k, l % 16]
    D = run(probe, 2, a, b)
    # A wrong lane layout gives errors of the order of the result itself. The
    # hardware's FP8 dot product is not exact: compare with the exact product
    # and with one whose subnormal inputs are flushed to zero, and bound the
    # error relative to sum |a| |b|.
    ftz = lambda X: np.where(np.abs(X) < 2.0 ** -6, 0.0, X)
    mag = np.abs(A) @ np.abs(B)
    e_exact = float(np.max(np.abs(D - A @ B) / mag))
    e_ftz = float(np.max(np.abs(D - ftz(A) @ ftz(B)) / mag))
    print(f"fp8 mfma: max error / sum|ab| exact {e_exact:.2e}, subnormals flushed {e_ftz:.2e}")
    assert min(e_exact, e_ftz) < 2e-3
    # normal inputs only
    okn = np.where(np.isfinite(tab) & (np.abs(tab) <= 8) & (np.abs(tab) >= 2.0 ** -6))[0]
    ca = rng.choice(okn, (16, 128)).astype(np.uint8)
    cb = rng.choice(okn, (128, 16)).astype(np.uint8)
    A, B = tab[ca], tab[cb]
    for l in range(64):
        for e in range(32):
            k = 32 * (l // 16) + e
            a[l, e] = ca[l % 16, k]
            b[l, e] = cb[k, l % 16]
    D = run(probe, 2, a, b)
    e_norm = float(np.max(np.abs(D - A @ B) / (np.abs(A) @ np.abs(B))))
    print(f"fp8 mfma, normal inputs: max error / sum|ab| {e_norm:.2e}")
    assert e_norm < 2e-3


def test_conversions(probe):
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(4000) * 3, rng.standard_normal(4000) * 1e-3,
                        [0.0, -0.0, 440.0, -440.0, 0.0625, 1.0625, 1.1875]]).astype(np.float32)
    if x.size % 2:
        x = np.append(x, np.float32(0.5))
    tab = e4m3_table()
    fin = np.where(np.isfinite(tab))[0]
    for xs in (1.0, 0.25, 8.0):
        xd = torch.from_numpy(x).cuda()
        f8 = torch.zeros(x.size, dtype=torch.uint8, device="cuda")
        bf = torch.zeros(x.size, dtype=torch.int16, device="cuda")
        assert probe.probe_cvt(xd.data_ptr(), x.size, xs, f8.data_ptr(), bf.data_ptr()) == 0
        got = tab[f8.cpu().numpy()]
        y = x.astype(np.float64) / xs
        keep = np.abs(y) <= 448
        # nearest representable value; at a tie both neighbours are acceptable here
        dist = np.abs(tab[fin][None, :] - y[keep][:, None])
        best = dist.min(1)
        assert np.all(np.abs(got[keep] - y[keep]) <= best + 1e-12)
    # bf16: round to nearest even
    u = x.view(np.uint32).astype(np.uint64)
    rne = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    assert np.array_equal(bf.cpu().numpy().view(np.uint16), rne)
