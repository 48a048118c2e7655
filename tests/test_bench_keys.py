"""The benchmark's kernel keys against the product kernels the library defines.

The roofline line and the committed rocprofv3 summaries find the FP32 product kernels
by name.  Every FP32 instantiation that the product launches, named the way rocprofv3
prints it, must map to its key, and no FP64 instantiation may.  The template parameter
lists are read from the kernel source, so a kernel that gains a parameter fails here
until its names below (and, if needed, the benchmark's prefixes) follow."""
import importlib.util
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCE = os.path.join(ROOT, "paper_1712_02443_amd", "csrc", "aim_kernels.hip")

# kernel -> (key, FP32 names as rocprofv3 prints them, FP64 names that must not map)
PRODUCT_KERNELS = {
    "k_gemm_bf16x3": ("macro_gemm", ["k_gemm_bf16x3"], []),
    "k_gemm_f32": ("macro_gemm", ["k_gemm_f32"], []),
    "k_project": ("project", ["k_project<float>"], ["k_project<double>"]),
    "k_fft4_y_fwd": ("fft_y_fwd", ["k_fft4_y_fwd<float, 20, 20, 9>", "k_fft4_y_fwd<float, 16, 24, 0>"],
                     ["k_fft4_y_fwd<double, 20, 20, 9>"]),
    "k_fft_y_fwd": ("fft_y_fwd", ["k_fft_y_fwd<float>"], ["k_fft_y_fwd<double>"]),
    "k_fft4_x": ("fft_x_conv", ["k_fft4_x<float, 20, 20, 9>", "k_fft4_x<float, 25, 32, 8>"],
                 ["k_fft4_x<double, 20, 20, 9>"]),
    "k_fft_x": ("fft_x_conv", ["k_fft_x<float, 0>"], ["k_fft_x<double, 0>"]),
    "k_fft4_y_inv": ("fft_y_inv", ["k_fft4_y_inv<float, 20, 20, 9>"], ["k_fft4_y_inv<double, 20, 20, 9>"]),
    "k_fft_y_inv": ("fft_y_inv", ["k_fft_y_inv<float>"], ["k_fft_y_inv<double>"]),
    "k_near_mfma": ("near_field", ["k_near_mfma<float, 1>", "k_near_mfma<float, 2>"],
                    ["k_near_mfma<double, 1>", "k_near_mfma<double, 2>"]),
    "k_near": ("near_field", ["k_near<float>"], ["k_near<double>"]),
    "k_interp": ("interp_d", ["k_interp<float, 0, 3>", "k_interp<float, 0, 2>"], ["k_interp<double, 0, 3>"]),
}


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def template_arity(src: str, kernel: str) -> int:
    """Number of template parameters of a __global__ kernel (0 for a plain function)."""
    launch = r"(?:__launch_bounds__\((?:[^()]|\([^()]*\))*\)\s*)?"
    m = re.search(r"(template\s*<([^>]*)>\s*)?__global__\s+void\s+" + launch + re.escape(kernel) + r"\s*\(", src)
    assert m, f"{kernel} is not defined in aim_kernels.hip"
    return 0 if m.group(1) is None else len([p for p in m.group(2).split(",") if p.strip()])


def arity_of_name(name: str) -> int:
    return 0 if "<" not in name else len(name[name.index("<") + 1:name.rindex(">")].split(","))


@pytest.fixture(scope="module")
def bench():
    return load_bench()


@pytest.mark.parametrize("kernel", sorted(PRODUCT_KERNELS))
def test_product_kernel_names_map_to_their_key(bench, kernel):
    src = open(SOURCE).read()
    key, fp32, fp64 = PRODUCT_KERNELS[kernel]
    n = template_arity(src, kernel)
    for name in fp32 + fp64:
        assert arity_of_name(name) == n, f"{name}: {kernel} takes {n} template parameters"
    for name in fp32:
        assert bench.kernel_key(name) == key, name
    for name in fp64:
        assert bench.kernel_key(name) == "", name


def test_other_kernels_have_no_key(bench):
    for name in ("k_gemm_f64", "k_transpose<float>", "k_extract_spectrum<float>", "k_interp<float, 1, 3>",
                 "k_interp<float, 2, 3>", "k_fft_x<float, 1>", "__amd_rocclr_copyBuffer"):
        assert bench.kernel_key(name) == "", name
