// Host-side argument checks and conversion of ABI structs to launch form.
#pragma once

#include <stddef.h>

#include <string>

#include "../../include/cloud.h"
#include "cloud_types.h"

namespace cloud {

// Records msg as this thread's last error and returns code.
int fail(int code, const std::string& msg);
void clear_error();

// Each returns CLOUD_OK or CLOUD_E_INVALID (with the message set).
int prepare_volume(const cloud_volume* v, DevVolume* out, int* dtype);
// Device bytes of v's base volume stored in `layout` (checks the dims).
int volume_layout_bytes(const cloud_volume* v, int layout, size_t* bytes);
int prepare_params(const cloud_params* p, const cloud_volume* v, DevParams* out);
int prepare_camera(const cloud_camera* c, int W, int H, DevCamera* out);
int check_image(int W, int H, long long views);

// The device allocation holding [p, p + bytes) must exist (device, managed or
// pinned host memory). Returns CLOUD_OK or CLOUD_E_INVALID naming `what`.
int check_span(const void* p, size_t bytes, const char* what);

size_t dtype_size(int dtype);

}  // namespace cloud
