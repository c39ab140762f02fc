"""FP64 CPU oracle of the musculoskeletal step -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package; the product path (the HIP library and its binding)
never does.
"""
from .oracle import Oracle, adam, bf16, build_oracle, mlp_forward, mlp_grad, oracle_lib_path  # noqa: F401
from .policy import policy_act, policy_obs, quat_to_rotvec, reference_targets  # noqa: F401
