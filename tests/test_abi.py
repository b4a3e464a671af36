"""Host-side checks of the C ABI: the built library loads and exports every
entry point that include/bpm.h declares, and the binding declares the same set.
No compute call is made (no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bpm.h")
LIB = os.path.join(ROOT, "paper_2601_06340_amd", "libbpm_hip.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(bpm_[a-z0-9_]+)\s*\(", src))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("bpm_plan_create", "bpm_propagate", "bpm_batch_submit", "bpm_poll"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in sorted(declared_functions()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2601_06340_amd import bpm
    assert set(bpm.SIGNATURES) == declared_functions()


def test_synth_module_holds_no_method_arithmetic():
    """The shared input module must not compute propagators, couplings or FFTs."""
    import io
    import tokenize
    path = os.path.join(ROOT, "paper_2601_06340_amd", "synth.py")
    code = " ".join(t.string for t in tokenize.generate_tokens(io.StringIO(open(path).read()).readline)
                    if t.type not in (tokenize.STRING, tokenize.COMMENT)).lower()
    for banned in ("fft", "jv", "bessel", "propagat", "oracle"):
        assert banned not in code, banned


def test_oracle_and_product_share_no_code():
    """The HIP sources never include or name the oracle, and vice versa."""
    csrc = os.path.join(ROOT, "paper_2601_06340_amd", "csrc")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "oracle" not in txt.lower(), f
    for f in ("bpm.py", "synth.py", "__init__.py", "build.py"):
        txt = open(os.path.join(ROOT, "paper_2601_06340_amd", f)).read()
        assert "import oracle" not in txt and "from oracle" not in txt, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_2601_06340_amd" not in txt.replace("paper_2601_06340_amd.synth", ""), f


def test_twiddle_schedule_matches_kernel_geometry():
    """The host-side twiddle schedule and the kernel's work split come from the
    same rule; a mismatch for some sizes once produced wrong transforms."""
    src = open(os.path.join(ROOT, "paper_2601_06340_amd", "csrc", "bpm_setup.hip")).read()
    body = src[src.index("inline int schedule_radices"):]
    body = body[:body.index("}")]
    assert "use_wave_groups" in body


def test_every_synthetic_workload_passes_descriptor_validation():
    """Every workload recipe produces descriptors the library accepts: without a
    GPU, plan creation gets past validation and stops at the device check."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present: covered by the GPU tests")
    from paper_2601_06340_amd import bpm, synth
    if not os.path.exists(bpm.LIB_PATH):
        pytest.skip("library not built")
    probs = [p for p, _ in synth.flat_bragg_scan(n_angles=2)]
    probs += [p for p, _ in synth.bent_laue(beams_per_radius=1)]
    probs += [p for p, _ in synth.disl_bragg_cores(2)]
    probs += [p for p, _ in synth.td_batch(n_comp=32)]
    probs += [r["problem"] for r in synth.serve_mix(n_req=300)]
    for p in probs:
        with pytest.raises(bpm.BpmError) as e:
            bpm.Plan(p)
        assert e.value.status == bpm.E_DEVICE, (p["nx"], p["nz"], p.get("kind"), str(e.value))


def test_tables_beyond_32_bit_offsets_are_refused_before_the_device():
    """A strain table or mask too large for the kernels' 32-bit byte offsets is
    BPM_E_UNSUPPORTED at validation (the table itself is not read)."""
    import numpy as np
    from paper_2601_06340_amd import bpm, synth
    if not os.path.exists(bpm.LIB_PATH):
        pytest.skip("library not built")
    nx, nz = 65536, 9000                       # FP32 table: 2.36e9 bytes
    seg = np.zeros((nz, 1, 2), np.int32)
    seg[:, 0, 1] = nx
    p = synth.base_problem(nx, nz, 0.1, 0.05, seg, precision="f32",
                           strain={"kind": "table", "u_table": np.zeros((1, nx))})
    with pytest.raises(bpm.BpmError) as e:
        bpm.Plan(p)
    assert e.value.status == bpm.E_UNSUPPORTED, str(e.value)


def test_3d_sizes_outside_the_built_kernels_are_refused_before_the_device():
    """3D envelopes take nx and ny powers of two with 256 <= nx <= 1024 and
    16 <= ny <= 256; other powers of two are BPM_E_UNSUPPORTED at validation
    (an nx that is no power of two is BPM_E_INVALID for every plan)."""
    import numpy as np
    from paper_2601_06340_amd import bpm, synth
    if not os.path.exists(bpm.LIB_PATH):
        pytest.skip("library not built")
    for nx, ny, want in ((128, 16, bpm.E_UNSUPPORTED), (2048, 16, bpm.E_UNSUPPORTED), (384, 16, bpm.E_INVALID),
                         (512, 8, bpm.E_UNSUPPORTED), (512, 512, bpm.E_UNSUPPORTED), (256, 48, bpm.E_UNSUPPORTED)):
        seg = np.zeros((4, ny, 1, 2), np.int32)
        seg[:, :, 0, 1] = nx
        p = synth.base_problem(nx, 4, 0.1, 0.05, seg, precision="f32")
        p["ny"], p["dy_um"] = ny, 0.2
        with pytest.raises(bpm.BpmError) as e:
            bpm.Plan(p)
        assert e.value.status == want, (nx, ny, str(e.value))


def test_coupling_step_beyond_the_series_bound_is_refused_before_the_device():
    """A plan whose coupling sub-step has |A^2 chih chihbar| above 100 or
    |A chi0| above 700 (A = b k dz / 2 cos theta_B, Eq. (9)-(12)) is
    BPM_E_INVALID at validation; just below the bound it passes validation.
    The marches weight the coupling by 0 outside the crystal, which needs
    finite coefficients: the bound guarantees them."""
    import math
    import numpy as np
    from paper_2601_06340_amd import bpm, synth
    if not os.path.exists(bpm.LIB_PATH):
        pytest.skip("library not built")
    nx = 256
    k = 2 * math.pi / synth.LAMBDA_UM
    c = math.sqrt(1 - (synth.LAMBDA_UM / (2 * synth.D_UM)) ** 2)

    def dz_for(y):   # order 1: b = 1, |A|^2 |chih| |chihb| = y
        return math.sqrt(y / (abs(synth.CHIH) ** 2)) * 2 * c / k

    import torch
    for y in (101.0, 1e4, 99.0):
        seg = synth.mask_x_slab(2, nx, 0.1, 0.0, nx * 0.1)
        p = synth.base_problem(nx, 2, 0.1, dz_for(y), seg, precision="f32")
        if y < 100.0:
            if torch.cuda.is_available():
                bpm.Plan(p).close()
                continue
            want = bpm.E_DEVICE   # past validation, stopped at the device check
        else:
            want = bpm.E_INVALID
        with pytest.raises(bpm.BpmError) as e:
            bpm.Plan(p)
        assert e.value.status == want and (want != bpm.E_INVALID or "coupling step" in str(e.value)), (y, str(e.value))
    # |A chi0| > 700 with chih = chihbar = 0
    seg = synth.mask_x_slab(2, nx, 0.1, 0.0, nx * 0.1)
    p = synth.base_problem(nx, 2, 0.1, 701.0 * 2 * c / (k * abs(synth.CHI0)), seg, precision="f32",
                           chih=0j, chihb=0j)
    with pytest.raises(bpm.BpmError) as e:
        bpm.Plan(p)
    assert e.value.status == bpm.E_INVALID and "coupling step" in str(e.value)
