"""MI355X-native batched musculoskeletal forward-dynamics step.

The compute path is the HIP library ``libms.so`` (C ABI in include/ms.h);
``ms`` binds it with ctypes and uses torch only for device memory and
streams. ``synth`` builds seeded synthetic models and excitations.
"""
