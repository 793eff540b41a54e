"""Host-side logic of bench.py: the byte model and the code hash that ties stored HBM
counters to the kernels they were taken on (no GPU)."""
import bench


def test_code_tokens_ignore_comments_and_layout():
    a = "int f(int x) {  // first\n    return x + 1; /* block\n comment */ }\n"
    b = "int f(int x) {\n  return x + 1;   }  // another comment\n"
    c = "int f(int x) { return x + 2; }"
    assert bench.code_tokens(a) == bench.code_tokens(b) == "int f(int x) { return x + 1; }"
    assert bench.code_tokens(c) != bench.code_tokens(a)


def test_source_hash_per_kernel_file():
    # the explicit kernels and the spectral kernels hash different files
    assert bench.source_hash("advance") == bench.source_hash("mu")
    assert bench.source_hash("dht_x") == bench.source_hash("tridiag_pair")
    assert bench.source_hash("advance") != bench.source_hash("dht_x")
    assert len(bench.source_hash("dht_x")) == 16


def test_kernel_bytes_model():
    nx, ny, nz = 128, 128, 128
    ni = nx * (ny - 2) * nz
    # a transform pass reads and writes three spectral fields of the interior rows
    assert bench.kernel_bytes("dht_x", nx, ny, nz) == 48 * ni
    # both flow residuals: omega, S and psi, three components each
    assert bench.kernel_bytes("resid_norm_flow", nx, ny, nz) == 72 * ni


def test_system_info_without_a_device():
    # every field is present; what cannot be read here (no GPU) is None, not an exception
    import torch
    info = bench.system_info(torch)
    assert set(info) == {"device", "arch", "compute_units", "hip", "torch", "rocm", "clocks"}
    assert info["torch"] == torch.__version__
    if not torch.cuda.is_available():
        assert info["device"] is None and info["compute_units"] is None


def test_more_than_one_gpu_is_refused():
    # one simulation per GPU on one GPU: --gpus above 1 (or a multi-rank launch) exits with
    # status 2 and says so, before touching a device
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py")] + args,
                           capture_output=True, text=True, timeout=120,
                           env=dict(os.environ, **env))
        assert r.returncode == 2, (args, env, r.stderr)
        assert "not supported" in r.stderr and r.stdout == ""
