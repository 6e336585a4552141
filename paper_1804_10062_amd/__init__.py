"""QuickMergesort on AMD Instinct MI355X (gfx950).

The sort itself runs in the HIP kernels of ``libqms.so`` (C ABI in
``include/qms.h``); ``qms`` is its thin ctypes binding and ``inputs`` the
seeded synthetic workloads.
"""
from .qms import (  # noqa: F401
    QMS_F32, QMS_U32, QmsError, Server, load_library, qms_get_tiles,
    qms_last_schedule, qms_profile_begin, qms_profile_end, qms_release_workspaces, qms_sort, qms_sort_batch,
    qms_sort_pairs,
)
