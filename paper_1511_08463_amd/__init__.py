"""MI355X (gfx950) phase-field fracture solver: HIP library + Python binding.

``fracture`` binds the C ABI of ``include/fracture.h`` (libfracture.so, built
by ``build.build()``); ``workloads`` holds the seeded synthetic inputs.
"""
