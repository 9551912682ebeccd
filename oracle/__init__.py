"""CPU oracle for the SDM collision-coalescence step.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path
(``paper_2103_17238_amd``) never does, and this package never imports the
product.  It shares no code with the HIP library.

``sdm_oracle.c`` holds the step itself (plain C, fp64, -ffp-contract=off);
``oracle.py`` is its ctypes wrapper and ``closed_form.py`` the analytic Golovin
solution and binning helpers used to pin it.
"""
from .oracle import (  # noqa: F401
    GOLOVIN,
    GEOMETRIC,
    ST_SUBSTEP_CAP,
    ST_GAMMA_CAP,
    OracleConfig,
    build,
    lib,
    philox4x32_10,
    philox_fill,
    phi_from_words,
    kernel_value,
    radius,
    terminal_velocity,
    scale_factor,
    pair_probability,
    gamma_from,
    update_pair,
    cell_order,
    pairs_for_order,
    step,
    moments,
    probe_mul_add,
    max_threads,
    pair_base,
    cell_adaptive_trace,
)
