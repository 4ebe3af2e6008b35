// bf_parquet.hip -- host side of the Parquet split-block filter
// (include/bf_parquet.h): creation as a sectorized 8 x 32-bit, k = 8,
// seed-0 filter whose kernels take the format's multipliers, its kernel
// table, and the format's bloom filter header in the Thrift compact
// protocol.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/bf_parquet.h"
#include "bf_internal.hpp"
#include "bf_registry.hpp"

namespace bfhip {

Registry& parquet_registry() {
  static Registry r{};
  return r;
}

void ensure_parquet_registry() {
  static std::once_flag once;
  std::call_once(once, [] { register_parquet(parquet_registry()); });
}

const Registry& kernel_table(bool parquet) {
  if (parquet) {
    ensure_parquet_registry();
    return parquet_registry();
  }
  ensure_registry();
  return registry();
}

namespace {

constexpr uint64_t kBlockBytes = 32;  // eight 32-bit words

bool valid_size(uint64_t num_bytes) {
  return num_bytes >= kBlockBytes && num_bytes % kBlockBytes == 0 && num_bytes / kBlockBytes <= (1ull << 32);
}

// Thrift compact protocol: a field header byte is (id delta << 4) | type.
constexpr uint8_t kTypeStop = 0;
constexpr uint8_t kTypeBoolTrue = 1;
constexpr uint8_t kTypeBoolFalse = 2;
constexpr uint8_t kTypeByte = 3;
constexpr uint8_t kTypeI16 = 4;
constexpr uint8_t kTypeI32 = 5;
constexpr uint8_t kTypeI64 = 6;
constexpr uint8_t kTypeDouble = 7;
constexpr uint8_t kTypeBinary = 8;
constexpr uint8_t kTypeList = 9;
constexpr uint8_t kTypeSet = 10;
constexpr uint8_t kTypeMap = 11;
constexpr uint8_t kTypeStruct = 12;

// A bounded reader over the header bytes; any overrun sets `bad`.
struct Reader {
  const uint8_t* p;
  uint64_t len;
  uint64_t pos = 0;
  bool bad = false;

  uint8_t byte() {
    if (pos >= len) {
      bad = true;
      return 0;
    }
    return p[pos++];
  }
  uint64_t varint() {
    uint64_t v = 0;
    for (int shift = 0; shift < 70; shift += 7) {
      const uint8_t b = byte();
      if (bad) return 0;
      v |= static_cast<uint64_t>(b & 0x7f) << shift;
      if ((b & 0x80) == 0) return v;
    }
    bad = true;
    return 0;
  }
  int64_t zigzag() {
    const uint64_t z = varint();
    return static_cast<int64_t>(z >> 1) ^ -static_cast<int64_t>(z & 1);
  }
  void skip_bytes(uint64_t n) {
    if (n > len - pos) {
      bad = true;
      return;
    }
    pos += n;
  }
  // Skips one value of a compact type (nesting bounded by depth).
  void skip(uint8_t type, int depth) {
    if (depth > 32) {
      bad = true;
      return;
    }
    switch (type) {
      case kTypeBoolTrue:
      case kTypeBoolFalse:
        return;  // a field's bool lives in its header
      case kTypeByte:
        byte();
        return;
      case kTypeI16:
      case kTypeI32:
      case kTypeI64:
        varint();
        return;
      case kTypeDouble:
        skip_bytes(8);
        return;
      case kTypeBinary:
        skip_bytes(varint());
        return;
      case kTypeList:
      case kTypeSet: {
        const uint8_t h = byte();
        uint64_t n = h >> 4;
        if (n == 15) n = varint();
        for (uint64_t i = 0; i < n && !bad; ++i) skip_element(h & 0x0f, depth + 1);
        return;
      }
      case kTypeMap: {
        const uint64_t n = varint();
        if (n == 0 || bad) return;
        const uint8_t kv = byte();
        for (uint64_t i = 0; i < n && !bad; ++i) {
          skip_element(kv >> 4, depth + 1);
          skip_element(kv & 0x0f, depth + 1);
        }
        return;
      }
      case kTypeStruct:
        skip_struct(depth + 1);
        return;
      default:
        bad = true;
    }
  }
  // An element of a list, set or map: a bool there takes a byte of its own.
  void skip_element(uint8_t type, int depth) {
    if (type == kTypeBoolTrue || type == kTypeBoolFalse)
      byte();
    else
      skip(type, depth);
  }
  void skip_struct(int depth) {
    while (!bad) {
      const uint8_t h = byte();
      if (bad || (h & 0x0f) == kTypeStop) return;
      if ((h >> 4) == 0) zigzag();  // long form: explicit field id
      skip(h & 0x0f, depth);
    }
  }
  // A union of empty structs (the header's algorithm, hash and
  // compression): the id of its struct field, 0 if it has none or is
  // malformed.
  int16_t union_id(int depth) {
    int16_t id = 0, found = 0;
    while (!bad) {
      const uint8_t h = byte();
      if (bad || (h & 0x0f) == kTypeStop) break;
      id = (h >> 4) ? static_cast<int16_t>(id + (h >> 4)) : static_cast<int16_t>(zigzag());
      if ((h & 0x0f) == kTypeStruct && found == 0) found = id;
      skip(h & 0x0f, depth);
    }
    return bad ? 0 : found;
  }
};

}  // namespace
}  // namespace bfhip

using namespace bfhip;

extern "C" {

bf_status bf_create_parquet(uint64_t num_bytes, bf_filter** out) {
  if (out == nullptr || !valid_size(num_bytes)) return BF_EINVAL;
  bf_filter* f = nullptr;
  const bf_status st = bf_create(num_bytes / kBlockBytes, 8, 32, 8, 0, &f);
  if (st != BF_OK) return st;
  f->salts = kSaltsParquet;
  *out = f;
  return BF_OK;
}

bf_status bf_create_parquet_in(void* d_words, uint64_t num_bytes, bf_filter** out) {
  if (out == nullptr || !valid_size(num_bytes)) return BF_EINVAL;
  bf_filter* f = nullptr;
  const bf_status st = bf_create_in(num_bytes / kBlockBytes, 8, 32, 8, 0, d_words, num_bytes, &f);
  if (st != BF_OK) return st;
  f->salts = kSaltsParquet;
  *out = f;
  return BF_OK;
}

bf_status bf_parquet_header(uint64_t num_bytes, uint8_t* out, uint64_t cap, uint64_t* len) {
  if (out == nullptr || len == nullptr || !valid_size(num_bytes) || num_bytes > 0x7fffffffull)
    return BF_EINVAL;
  uint8_t h[24];
  uint64_t n = 0;
  h[n++] = (1 << 4) | kTypeI32;  // field 1 numBytes: i32, zigzag varint
  uint64_t z = num_bytes << 1;
  while (z >= 0x80) {
    h[n++] = static_cast<uint8_t>(z | 0x80);
    z >>= 7;
  }
  h[n++] = static_cast<uint8_t>(z);
  // fields 2, 3, 4 (algorithm, hash, compression): unions whose field 1
  // (BLOCK, XXHASH, UNCOMPRESSED) is an empty struct
  for (int f = 0; f < 3; ++f) {
    h[n++] = (1 << 4) | kTypeStruct;
    h[n++] = (1 << 4) | kTypeStruct;
    h[n++] = kTypeStop;  // end of the empty struct
    h[n++] = kTypeStop;  // end of the union
  }
  h[n++] = kTypeStop;
  *len = n;
  if (cap < n) return BF_EINVAL;
  for (uint64_t i = 0; i < n; ++i) out[i] = h[i];
  return BF_OK;
}

bf_status bf_parquet_parse_header(const uint8_t* blob, uint64_t len, uint64_t* num_bytes,
                                  uint64_t* header_len) {
  if (blob == nullptr || num_bytes == nullptr || header_len == nullptr) return BF_EINVAL;
  Reader r{blob, len};
  int64_t nbytes = -1;
  int16_t algorithm = -1, hash = -1, compression = -1, id = 0;
  while (!r.bad) {
    const uint8_t h = r.byte();
    if (r.bad || (h & 0x0f) == kTypeStop) break;
    id = (h >> 4) ? static_cast<int16_t>(id + (h >> 4)) : static_cast<int16_t>(r.zigzag());
    const uint8_t type = h & 0x0f;
    if (id == 1 && type == kTypeI32) {
      nbytes = r.zigzag();
    } else if (id >= 2 && id <= 4 && type == kTypeStruct) {
      const int16_t v = r.union_id(0);
      (id == 2 ? algorithm : id == 3 ? hash : compression) = v;
    } else {
      r.skip(type, 0);
    }
  }
  if (r.bad || nbytes <= 0 || nbytes % 32 != 0 || algorithm <= 0 || hash <= 0 || compression <= 0)
    return BF_EINVAL;
  if (algorithm != 1 || hash != 1 || compression != 1) return BF_EUNSUPPORTED;
  *num_bytes = static_cast<uint64_t>(nbytes);
  *header_len = r.pos;
  return BF_OK;
}

}  // extern "C"
