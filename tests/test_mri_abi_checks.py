"""Argument checks of the multicoil MRI C-ABI (include/skei_mri.h).  Every
case here is refused before anything touches a device, so this runs without
a GPU (the pointers are placeholders that are never dereferenced)."""
import ctypes

from paper_2411_05771_amd import capi

P = ctypes.c_void_p(16)   # a non-null placeholder, never dereferenced
EINVAL, ERANGE = -1, -4


def lib():
    return capi.lib()


def test_transform_sizes_and_pointers(hiplib):
    for n in (0, 1, 2, 3, 12, 100, 2048, 4096):   # not a power of two in [4, 1024]
        assert lib().skei_mri_fwd(P, 2, n, P, 1, P, None, P, None) == EINVAL, n
        assert lib().skei_mri_adj(P, 2, n, P, 1, P, None, P, P, None) == EINVAL, n
    assert lib().skei_mri_fwd(P, 0, 16, P, 1, P, None, P, None) == EINVAL      # no coils
    assert lib().skei_mri_fwd(P, 2, 16, P, 0, P, None, P, None) == EINVAL      # no images
    assert lib().skei_mri_fwd(None, 2, 16, P, 1, P, None, P, None) == EINVAL   # null maps
    assert lib().skei_mri_adj(P, 2, 16, P, 1, P, None, P, None, None) == EINVAL   # no scratch
    assert lib().skei_mri_fwd(P, 1 << 20, 16, P, 1 << 12, P, None, P, None) == ERANGE   # grid beyond 2^31


def test_work_bytes(hiplib):
    lib().skei_mri_work_bytes.restype = ctypes.c_size_t
    assert lib().skei_mri_work_bytes(15, 128, 3) == 3 * 15 * 128 * 128 * 8
    assert lib().skei_mri_work_bytes(0, 128, 3) == 0


def test_coil_kernel_checks(hiplib):
    assert lib().skei_coil_mix(P, 0, 4, P, 1, ctypes.c_longlong(16), P, None) == EINVAL
    assert lib().skei_coil_mix(P, 1025, 4, P, 1, ctypes.c_longlong(16), P, None) == ERANGE
    assert lib().skei_coil_mix(P, 4, 1025, P, 1, ctypes.c_longlong(16), P, None) == ERANGE
    assert lib().skei_coil_covariance(P, 65, ctypes.c_longlong(16), P, None) == ERANGE
    assert lib().skei_coil_covariance(P, 4, ctypes.c_longlong(1), P, None) == EINVAL
    assert lib().skei_coil_weights(None, 4, 16, P, None) == EINVAL
