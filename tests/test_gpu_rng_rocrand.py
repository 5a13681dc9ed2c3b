"""The reference Philox4x32-10 against a second, independent implementation:
rocRAND's PHILOX4_32_10 device generator.  With seed s its i-th block of four
32-bit words is Philox4x32-10 of the counter (i, 0, 0, 0) under the key
(low 32 bits of s, high 32 bits of s).  rocRAND needs a HIP device, so the
check runs with the GPU tests; the known-answer vectors of the round function
are checked on the CPU."""
import ctypes as C
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

_ROCRAND = "/opt/rocm/lib/librocrand.so"
_PHILOX4_32_10 = 404  # rocrand_rng_type


@pytest.mark.skipif(not os.path.exists(_ROCRAND), reason="rocRAND not installed")
@pytest.mark.parametrize("seed", [0, 0x0123456789ABCDEF, 0xFFFFFFFF00000001])
def test_reference_philox_equals_rocrand(oracle_mod, seed):
    import torch

    lib = C.CDLL(_ROCRAND)
    gen = C.c_void_p()
    assert lib.rocrand_create_generator(C.byref(gen), _PHILOX4_32_10) == 0
    try:
        assert lib.rocrand_set_seed(gen, C.c_ulonglong(seed)) == 0
        n_blocks = 1024
        buf = torch.zeros(4 * n_blocks, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        assert lib.rocrand_generate(gen, C.c_void_p(buf.data_ptr()), C.c_size_t(4 * n_blocks)) == 0
        torch.cuda.synchronize()
        got = buf.cpu().numpy().view(np.uint32).reshape(n_blocks, 4)
    finally:
        lib.rocrand_destroy_generator(gen)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    want = np.stack([oracle_mod.philox([i, 0, 0, 0], key) for i in range(n_blocks)])
    assert np.array_equal(got, want)
