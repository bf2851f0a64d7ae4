import numpy as np
import torch

from oracle.quant import to_bf16, to_f32


def test_bf16_matches_torch_cast():
    r = np.random.default_rng(0)
    a = np.concatenate([r.standard_normal(10000) * 10.0 ** r.integers(-8, 8, 10000),
                        # exact ties: float32 patterns with low half 0x8000
                        (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(np.float64)])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(to_bf16(a), ref)


def test_f32_rounding():
    a = np.array([1.0 + 2.0 ** -30, 1.0 / 3.0])
    np.testing.assert_array_equal(to_f32(a), a.astype(np.float32).astype(np.float64))
    assert to_f32(a)[0] == 1.0
