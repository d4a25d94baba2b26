"""The matrix-unit arithmetic the measured refinement bound rests on (needs the GPU).

Every code bit must be the sign of the exact projection outside the stated bound (Sec. 2.1),
so the bound's error model must cover what the matrix instructions really do.  Each test
runs single instructions through ace_mfma_probe on hand-built operands and compares D with
the exact value of C + A B (Python fractions):
  - FP32 16x16x4: products are exact and are added to the accumulator one after another in
    k order, each sum rounded to nearest even; over a chain of I instructions the error is
    within gamma_{4I}(2^-24) sum |p|  (the library's h = DP + 4).
  - BF16 16x16x32: each group of 8 consecutive k is aligned to its largest product and cut
    below 2^-24 of it; group sums enter the accumulator rounded to nearest; the error of a
    chain is within (4 + 2I) 2^-23 sum |p| (the library's main-chain term).
  - e4m3 16x16x128: a k-group loses less than 2^-10 of its largest product and the group
    sums enter the accumulator rounded to nearest; the error of a chain is within
    (2^-9 + 8I 2^-24) sum |p| (the library's term, twice the in-group loss).
Adversarial operands put many products just below each model's cut-off beside a large one,
with the same sign, so that a wider alignment window or fewer kept bits than the model
assumes would push the error past the bound.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _probe(kind, A, B, C):
    from paper_1706_06664_amd import mfma_probe
    return mfma_probe(kind, A, B, C)


# ---- number formats ------------------------------------------------------------------------

def bf16_bits(x):
    """Round-to-nearest-even FP32 -> BF16 bits (finite x)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_value(bits):
    return (np.asarray(bits, np.uint32) << 16).view(np.float32).astype(np.float64)


def e4m3_value(code):
    """Value of an OCP e4m3 code (bias 7, no infinities; 0x7F / 0xFF are NaN)."""
    code = np.asarray(code, np.int64)
    s = np.where(code & 0x80, -1.0, 1.0)
    E = (code >> 3) & 0xF
    M = code & 7
    v = np.where(E == 0, M / 8.0 * 2.0 ** -6, (1 + M / 8.0) * 2.0 ** (E - 7))
    return s * v


def e4m3_code(v):
    """Code of an e4m3-representable value (exact; raises otherwise)."""
    table = {float(e4m3_value(c)): c for c in range(256) if (c & 0x7F) != 0x7F}
    table[0.0] = 0
    out = np.vectorize(lambda x: table[float(x)])(np.asarray(v, np.float64))
    return out.astype(np.uint8)


# ---- exact reference -----------------------------------------------------------------------

def exact_chain(As, Bs, C0=None):
    """Exact sum_i A_i B_i (+ C0) per output and sum |products|, as Fractions [16][16]."""
    ex = [[Fraction(0) if C0 is None else Fraction(float(C0[r, c])) for c in range(16)] for r in range(16)]
    ab = [[Fraction(0) for _ in range(16)] for _ in range(16)]
    for A, B in zip(As, Bs):
        fa = [[Fraction(float(v)) for v in row] for row in A]
        fb = [[Fraction(float(v)) for v in row] for row in B.T]
        for r in range(16):
            for c in range(16):
                s = Fraction(0)
                t = Fraction(0)
                for x, y in zip(fa[r], fb[c]):
                    if x and y:
                        p = x * y
                        s += p
                        t += abs(p)
                ex[r][c] += s
                ab[r][c] += t
    return ex, ab


def max_ratio(D, ex, bound):
    """max over outputs of |D - exact| / bound(r, c); bound(r, c) > 0."""
    worst = 0.0
    for r in range(16):
        for c in range(16):
            err = abs(Fraction(float(D[r, c])) - ex[r][c])
            worst = max(worst, float(err / bound(r, c)))
    return worst


def gamma(n, u):
    return Fraction(n) * u / (1 - Fraction(n) * u)


U24 = Fraction(1, 2 ** 24)
U23 = Fraction(1, 2 ** 23)


def run_chain(kind, As, Bs, to_operand):
    """D after I instructions, each taking the previous D as its accumulator (C0 = 0)."""
    D = np.zeros((16, 16), np.float32)
    for A, B in zip(As, Bs):
        D = _probe(kind, to_operand(A), to_operand(B), D)
    return D


# ---- FP32 ----------------------------------------------------------------------------------

def _fp32_case(c, pairs):
    """C = c everywhere; k-th product of every output is a_k * b_k."""
    A = np.zeros((16, 4), np.float32)
    B = np.zeros((4, 16), np.float32)
    for k, (a, b) in enumerate(pairs):
        A[:, k] = a
        B[k, :] = b
    return A, B, np.full((16, 16), c, np.float32)


@pytest.mark.parametrize("name,c,pairs,want", [
    # the product (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24 is not rounded before it meets C
    ("exact_product", -1.0, [(1 + 2 ** -12, 1 + 2 ** -12)], 2 ** -11 + 2 ** -24),
    # 1 + u + u with u = 2^-24: each sum is a tie that rounds to even -> 1 (not 1 + 2^-23)
    ("sequential_ties_to_even", 1.0, [(2 ** -12, 2 ** -12), (2 ** -12, 2 ** -12)], 1.0),
    # u + u + 1 (products in k order) keeps both units: 1 + 2^-23
    ("k_order", 0.0, [(2 ** -12, 2 ** -12), (2 ** -12, 2 ** -12), (1.0, 1.0)], 1.0 + 2 ** -23),
    # 2^30 + 1 - 2^30: the 1 is rounded away before the cancellation
    ("cancellation_after_rounding", 0.0, [(2 ** 15, 2 ** 15), (1.0, 1.0), (2 ** 15, -2 ** 15)], 0.0),
])
def test_fp32_exact_products_sequential_rne(name, c, pairs, want):
    A, B, C = _fp32_case(c, pairs)
    D = _probe("fp32", A, B, C)
    assert np.all(D == np.float32(want)), (name, np.unique(D))


@pytest.mark.parametrize("I,seed,adversarial", [(1, 1, False), (16, 2, False), (128, 3, False),
                                                (16, 4, True), (128, 5, True)])
def test_fp32_chain_within_bound(I, seed, adversarial):
    rng = np.random.default_rng(seed)
    As, Bs = [], []
    for i in range(I):
        A = rng.standard_normal((16, 4)).astype(np.float32)
        B = rng.standard_normal((4, 16)).astype(np.float32)
        if adversarial:
            # long cancelling chains: each product pair nearly cancels, and the running sum
            # stays large against the residuals
            A[:, 1] = A[:, 0] * np.float32(1 + 2 ** -20)
            B[1, :] = -B[0, :]
            A[:, 3] = np.float32(2 ** -13) * A[:, 2]
        As.append(A)
        Bs.append(B)
    D = run_chain("fp32", As, Bs, lambda x: x)
    ex, ab = exact_chain(As, Bs)
    g = gamma(4 * I, U24)
    ratio = max_ratio(D, ex, lambda r, c: g * ab[r][c])
    print(f"fp32 I={I} adversarial={adversarial}: max |err| / bound = {ratio:.4f}", flush=True)
    assert ratio <= 1.0


# ---- BF16 ----------------------------------------------------------------------------------

T_BF16 = 2.0 ** -12 * (1 - 2.0 ** -7)   # t^2 just below 2^-24, so t^2 falls under the cut of a product of 1


def _bf16_case(tiny_positions, big_positions=(0,), c=0.0):
    A = np.zeros((16, 32), np.float32)
    for k in big_positions:
        A[:, k] = 1.0
    for k in tiny_positions:
        A[:, k] = T_BF16
    B = np.ascontiguousarray(A.T)
    return A, B, np.full((16, 16), c, np.float32)


def test_bf16_groups_of_eight():
    # seven products just below 2^-24 beside a 1 in the same group of 8 are cut away
    A, B, C = _bf16_case(range(1, 8))
    D = _probe("bf16", bf16_bits(A), bf16_bits(B), C)
    assert np.all(D == 1.0), np.unique(D)
    # the same eight tiny products in the next group keep their value: that group is aligned
    # to its own largest product, and its sum 8 t^2 enters the accumulator rounded to nearest
    A, B, C = _bf16_case(range(8, 16))
    D = _probe("bf16", bf16_bits(A), bf16_bits(B), C)
    assert np.all(D == np.float32(1 + 2 ** -21)), np.unique(D)


@pytest.mark.parametrize("tiny", [range(1, 8), range(1, 32), [1, 2, 3, 9, 17, 25, 31]])
def test_bf16_truncation_within_bound(tiny):
    """Tiny products next to a single 1: with 8-product groups only the 1's group loses
    them (error < 7 x 2^-24); one alignment over all 32 products would lose all 31 and
    break the bound 4u sum|p| + 2u (|C| + sum|p|)."""
    A, B, C = _bf16_case(tiny)
    D = _probe("bf16", bf16_bits(A), bf16_bits(B), C)
    Av, Bv = bf16_value(bf16_bits(A)), bf16_value(bf16_bits(B))
    ex, ab = exact_chain([Av], [Bv])
    ratio = max_ratio(D, ex, lambda r, c: 4 * U23 * ab[r][c] + 2 * U23 * ab[r][c])
    print(f"bf16 tiny positions {list(tiny)}: max |err| / bound = {ratio:.4f}", flush=True)
    assert ratio <= 1.0


@pytest.mark.parametrize("I,seed,mode", [(1, 11, "normal"), (8, 12, "normal"), (64, 13, "normal"),
                                         (8, 14, "cut"), (64, 15, "cut"), (8, 16, "big_c")])
def test_bf16_chain_within_bound(I, seed, mode):
    """Chains of I instructions against the library's main-chain term (4 + 2I) u sum|p|
    (u = 2^-23).  'cut': every group of every instruction holds one large product and seven
    of the same sign just below its cut, at a random scale per group.  'big_c': the chain
    starts from a large accumulator, so the roundings of the group sums dominate; it is
    checked per instruction against 4u sum|p| + 2u (|C| + sum|p|)."""
    rng = np.random.default_rng(seed)
    As, Bs = [], []
    for i in range(I):
        if mode == "cut":
            A = np.zeros((16, 32), np.float32)
            B = np.zeros((32, 16), np.float32)
            for g in range(4):
                sa = 2.0 ** rng.integers(-8, 8, size=16)
                sb = 2.0 ** rng.integers(-8, 8, size=16)
                A[:, 8 * g] = sa
                B[8 * g, :] = sb
                for k in range(8 * g + 1, 8 * g + 8):
                    A[:, k] = sa * T_BF16
                    B[k, :] = sb * T_BF16
        else:
            A = rng.standard_normal((16, 32)).astype(np.float32)
            B = rng.standard_normal((32, 16)).astype(np.float32)
        As.append(bf16_value(bf16_bits(A)))
        Bs.append(bf16_value(bf16_bits(B)))
    if mode == "big_c":
        C = np.full((16, 16), 2.0 ** 20, np.float32) * rng.choice([-1, 1], size=(16, 16)).astype(np.float32)
        worst = 0.0
        for A, B in zip(As, Bs):
            D = _probe("bf16", bf16_bits(A), bf16_bits(B), C)
            ex, ab = exact_chain([A], [B], C0=C)
            worst = max(worst, max_ratio(D, ex, lambda r, c: 4 * U23 * ab[r][c] + 2 * U23 * (
                abs(Fraction(float(C[r, c]))) + ab[r][c])))
            C = D
        print(f"bf16 big accumulator, {I} instructions: max |err| / bound = {worst:.4f}", flush=True)
        assert worst <= 1.0
        return
    D = run_chain("bf16", As, Bs, bf16_bits)
    ex, ab = exact_chain(As, Bs)
    h = 4 + 2 * I
    ratio = max_ratio(D, ex, lambda r, c: h * U23 * ab[r][c])
    print(f"bf16 I={I} {mode}: max |err| / bound = {ratio:.4f}", flush=True)
    assert ratio <= 1.0


# ---- e4m3 ----------------------------------------------------------------------------------

def _e4m3_pair(s):
    """A big e4m3 value g (product g^2) and two e4m3 values whose product is 1.875 2^-s g^2,
    just below 2^{1-s} of the big product.  g grows past 1 only where the tiny product
    would fall below what two e4m3 values can make."""
    for eg in range(0, 9):
        for ea in range(-6, 9):
            b = 2.0 ** (2 * eg - s - ea)
            if 2.0 ** -9 <= b <= 448:
                return 2.0 ** eg, 1.875 * 2.0 ** ea, b
    raise ValueError(s)


def _e4m3_case(big_positions, tiny_positions, s):
    g, a_t, b_t = _e4m3_pair(s)
    A = np.zeros((16, 128))
    for k in big_positions:
        A[:, k] = g
    for k in tiny_positions:
        A[:, k] = a_t
    B = np.zeros((128, 16))
    for k in big_positions:
        B[k, :] = g
    for k in tiny_positions:
        B[k, :] = b_t
    return A, B


@pytest.mark.parametrize("s", [9, 10, 11, 12, 13, 14, 16])
@pytest.mark.parametrize("layout", ["one_big_per_8", "one_big_in_all"])
def test_e4m3_in_group_loss_within_bound(s, layout):
    """A product of 1 beside tiny products of 1.875 2^-s, all positive: 'one_big_per_8'
    puts a 1 at every 8th position (every group of 8 or more consecutive k holds one),
    'one_big_in_all' a single 1 for all 128.  The loss must stay within the e4m3 term
    (2^-9 + 8 2^-24) sum |p|: a group that kept fewer bits, or one alignment over all 128
    products, would break it."""
    if layout == "one_big_per_8":
        big = list(range(0, 128, 8))
        tiny = [k for k in range(128) if k % 8]
    else:
        big = [0]
        tiny = list(range(1, 128))
    A, B = _e4m3_case(big, tiny, s)
    D = _probe("e4m3", e4m3_code(A), e4m3_code(B), np.zeros((16, 16), np.float32))
    ex, ab = exact_chain([A], [B])
    bound = Fraction(1, 2 ** 9) + 8 * U24
    ratio = max_ratio(D, ex, lambda r, c: bound * ab[r][c])
    rel = float(abs(Fraction(float(D[0, 0])) - ex[0][0]) / ab[0][0])
    print(f"e4m3 {layout} s={s}: loss / sum|p| = 2^{math.log2(rel) if rel else -math.inf:.2f}, "
          f"ratio to bound {ratio:.4f}", flush=True)
    assert ratio <= 1.0


@pytest.mark.parametrize("I,seed,heavy", [(1, 21, False), (8, 22, False), (32, 23, False), (32, 24, True)])
def test_e4m3_chain_within_bound(I, seed, heavy):
    """Random finite e4m3 operands (uniform over the codes, or heavy-tailed Student-t values
    rounded to e4m3) through chains of I instructions, against (2^-9 + 8 I 2^-24) sum |p|."""
    import torch
    rng = np.random.default_rng(seed)
    finite = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    As, Bs = [], []
    for i in range(I):
        if heavy:
            # clipped to the finite range first: the cast turns values past 448 into NaN
            A = torch.from_numpy(np.clip(rng.standard_t(3, (16, 128)) * 16, -448, 448)
                                 .astype(np.float32)).to(torch.float8_e4m3fn)
            B = torch.from_numpy(np.clip(rng.standard_t(3, (128, 16)) * 16, -448, 448)
                                 .astype(np.float32)).to(torch.float8_e4m3fn)
            A = e4m3_value(A.view(torch.uint8).numpy())
            B = e4m3_value(B.view(torch.uint8).numpy())
        else:
            A = e4m3_value(rng.choice(finite, (16, 128)))
            B = e4m3_value(rng.choice(finite, (128, 16)))
        As.append(A)
        Bs.append(B)
    D = run_chain("e4m3", As, Bs, e4m3_code)
    ex, ab = exact_chain(As, Bs)
    bound = Fraction(1, 2 ** 9) + 8 * I * U24
    ratio = max_ratio(D, ex, lambda r, c: bound * ab[r][c] if ab[r][c] else Fraction(1))
    print(f"e4m3 I={I} heavy={heavy}: max |err| / bound = {ratio:.4f}", flush=True)
    assert ratio <= 1.0


def test_probe_rejects_bad_arguments():
    from paper_1706_06664_amd import load_library
    lib = load_library()
    z = np.zeros(2048, np.uint8)
    f = np.zeros(256, np.float32)
    assert lib.ace_mfma_probe(3, z.ctypes.data, z.ctypes.data, f.ctypes.data, f.ctypes.data, 0) == 1
    assert lib.ace_mfma_probe(0, None, z.ctypes.data, f.ctypes.data, f.ctypes.data, 0) == 1
