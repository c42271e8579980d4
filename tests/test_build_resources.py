"""Register and scratch budget of the hot kernels, from the compiler's resource-usage
report of the last build (no GPU).

The step and env kernels run one world's whole step per team with everything inlined
into the kernel: 128 VGPRs for four waves per SIMD, and a small private segment for
spills.  A per-world driver left as a real call has a stack frame of several hundred
bytes per lane (measured: 580 B and 35 % lower throughput), which these bounds catch.
The step kernel's bound also keeps its spill area (bytes per lane x 64 lanes x 4096
resident waves of the 8192-world quadruped launch) within the chip's L2: at 128 B per
lane it outgrew it and the spills reached HBM (1.3 GB written per launch instead of
16 MB).
"""
import pytest

from paper_2502_08844_amd import build

# instantiations without / with fourth-order Runge-Kutta groups, and the one that also
# solves elliptic-cone models
STEP = "_ZN3mjh15mjh_step_kernelILb0ELb0EEEvPKNS_8DevGroupEPKNS_7DevTaskEii"
STEP_RK = "_ZN3mjh15mjh_step_kernelILb1ELb0EEEvPKNS_8DevGroupEPKNS_7DevTaskEii"
STEP_CONE = "_ZN3mjh15mjh_step_kernelILb1ELb1EEEvPKNS_8DevGroupEPKNS_7DevTaskEii"
# env kernel: plain, with per-world randomised parameters, with Runge-Kutta
ENV = "_ZN3mjh14mjh_env_kernelILb0ELb0EEEvPKNS_8DevGroupEPKNS_7DevTaskENS_7EnvArgsEii"
ENV_DR = "_ZN3mjh14mjh_env_kernelILb0ELb1EEEvPKNS_8DevGroupEPKNS_7DevTaskENS_7EnvArgsEii"
ENV_RK = "_ZN3mjh14mjh_env_kernelILb1ELb0EEEvPKNS_8DevGroupEPKNS_7DevTaskENS_7EnvArgsEii"


@pytest.fixture(scope="module")
def usage():
    u = build.resource_usage()
    if u is None:
        pytest.skip("no build report yet (run the build first)")
    return u


@pytest.mark.parametrize("kernel,scratch_max", [(STEP, 16), (STEP_RK, 24), (STEP_CONE, 56),
                                                (ENV, 96), (ENV_DR, 128), (ENV_RK, 112)])
def test_hot_kernels_fit_four_waves_with_small_scratch(usage, kernel, scratch_max):
    k = usage[kernel]
    assert k["VGPRs"] <= 128 and k["Occupancy"] >= 4
    assert k["ScratchSize"] <= scratch_max, k


@pytest.mark.parametrize("kernel", [STEP])
def test_pyramid_step_kernels_spill_no_vgpr(usage, kernel):
    """The Newton loop's helpers re-derive their LDS base and lane from an opaque zero;
    without it the compiler hoisted their address arithmetic out of the iteration loop
    and spilled 31 VGPRs of the plain step kernel."""
    assert usage[kernel]["VGPRsSpill"] == 0, usage[kernel]
